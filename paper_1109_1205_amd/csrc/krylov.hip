// Krylov engine: Lanczos recursion (Eq. (recursion)), tridiagonal T
// (Eq. (tmatrix)) and its eigen-decomposition (Eq. (tdiag)), Ritz vectors
// (Eq. (eigen)), the ground state (Sec. 2) and the short-iterative-Lanczos
// step psi -> beta0 V Q exp(-i Lambda dt) Q^T e_1 (Eqs. (newstate),
// (udelta)).
//
// Storage: Lanczos vectors are kept unnormalised, v_k = s_k x_k, with the
// scale s_k = 1/b_k folded into the next kernel that reads x_k, so no
// separate normalisation pass over HBM is needed.  Every reduction writes
// one partial per block; a one-block finaliser sums them in a fixed order
// (results are reproducible run to run) and updates the per-column
// scalars.  A batch of ncol independent recursions (own a_k, b_k, T) runs
// in the same launches.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "kgf_internal.h"

namespace kgf {

namespace {

// per-column scalar block (doubles)
constexpr int kOffA = 0;                   // a[0..127]
constexpr int kOffB = 128;                 // b[0..128]
constexpr int kOffS = 258;                 // s[0..128]
constexpr int kOffBeta0 = 388;
constexpr int kOffSmax = 389;
constexpr int kOffCoef = 390;              // complex coef[0..128] (re, im)
constexpr int kScalStride = 648;
static_assert(kMaxKrylov <= 128 && kOffCoef % 2 == 0 && kScalStride % 2 == 0, "per-column scalar layout");
static_assert(kOffB == kScalOffB && kOffS == kScalOffS, "scalar offsets shared with the H.v kernels");

constexpr int kDotChunk = 8;               // vectors per multi-dot chunk

struct Slots {
    // slot(k, c) = k == 0 ? s0 + c * s0_col : X + (k - 1) * x_slot + c * x_col
    double2* s0;
    int64_t s0_col;
    double2* X;
    int64_t x_slot;
    int64_t x_col;
    __host__ __device__ double2* at(int k, int c) const {
        return k == 0 ? s0 + c * s0_col : X + (int64_t)(k - 1) * x_slot + c * x_col;
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// block sum in a fixed order; valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

int red_blocks(int64_t D) {
    int64_t nb = (D + kThreads * 4 - 1) / (kThreads * 4);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return (int)nb;
}

// ---------------------------------------------------------------------------
// streaming kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_norm2(const double2* __restrict__ X, int64_t col,
                                                    int64_t D, double* __restrict__ part) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.y;
    const double2* x = X + c * col;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 z = x[i];
        acc = fma(z.x, z.x, acc);
        acc = fma(z.y, z.y, acc);
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s;
}

// y_c -= a_k s_k x_c ; part = ||y_c||^2   (a_k, s_k at fa/fs + c * stride)
typedef double dbl2v __attribute__((ext_vector_type(2)));
// nontemporal load of a value read once (does not displace reused data)
__device__ __forceinline__ double2 ld_once(const double2* p) {
    const dbl2v v = __builtin_nontemporal_load(reinterpret_cast<const dbl2v*>(p));
    return make_double2(v.x, v.y);
}

__global__ __launch_bounds__(kThreads) void k_update(Slots sl, int k, const double* __restrict__ fa,
                                                     const double* __restrict__ fs, int stride,
                                                     int64_t D, double* __restrict__ part) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.y;
    const double f = fa[(int64_t)c * stride] * fs[(int64_t)c * stride];
    const double2* x = sl.at(k, c);
    double2* y = sl.at(k + 1, c);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 z = ld_once(x + i), w = y[i];
        w.x = fma(-f, z.x, w.x);
        w.y = fma(-f, z.y, w.y);
        y[i] = w;
        acc = fma(w.x, w.x, acc);
        acc = fma(w.y, w.y, acc);
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s;
}

// h_j = <s_j x_j, y> for j in chunk blockIdx.z (Gram-Schmidt coefficients);
// part layout [c][j][blk] with nj_total coefficient slots per column
__global__ __launch_bounds__(kThreads) void k_multidot(Slots sl, int ky, int nj,
                                                       const double* __restrict__ scal,
                                                       const double* __restrict__ gs_s,
                                                       int64_t D, double* __restrict__ part) {
    __shared__ double sh[kThreads / 64][2 * kDotChunk];
    const int c = blockIdx.y;
    const int j0 = blockIdx.z * kDotChunk;
    const int nloc = nj - j0 < kDotChunk ? nj - j0 : kDotChunk;
    const double2* y = sl.at(ky, c);
    double ar[kDotChunk], ai[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) ar[q] = ai[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 w = y[i];
#pragma unroll
        for (int q = 0; q < kDotChunk; ++q) {
            if (q < nloc) {
                const double2 z = sl.at(j0 + q, c)[i];
                ar[q] = fma(z.x, w.x, fma(z.y, w.y, ar[q]));
                ai[q] = fma(z.x, w.y, fma(-z.y, w.x, ai[q]));
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
        double r = wave_sum(ar[q]);
        double im = wave_sum(ai[q]);
        if (lane == 0) {
            sh[wv][2 * q] = r;
            sh[wv][2 * q + 1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nloc) {
        const int q = threadIdx.x >> 1, reim = threadIdx.x & 1;
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w][threadIdx.x];
        const int j = j0 + q;
        const double scale = gs_s ? gs_s[j] : scal[(int64_t)c * kScalStride + kOffS + j];
        part[(((int64_t)c * nj + j) * 2 + reim) * gridDim.x + blockIdx.x] = s * scale;
    }
}

// y -= sum_j h_j s_j x_j ; part = ||y||^2 .  h from hvec[c][j] (complex).
__global__ __launch_bounds__(kThreads) void k_multiaxpy(Slots sl, int ky, int nj,
                                                        const double* __restrict__ scal,
                                                        const double* __restrict__ gs_s,
                                                        const double2* __restrict__ hvec,
                                                        int64_t D, double* __restrict__ part) {
    extern __shared__ double2 sw[];
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.y;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        const double s = gs_s ? gs_s[j] : scal[(int64_t)c * kScalStride + kOffS + j];
        double2 h = hvec[(int64_t)c * nj + j];
        sw[j] = make_double2(h.x * s, h.y * s);
    }
    __syncthreads();
    double2* y = sl.at(ky, c);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 w = y[i];
        for (int j = 0; j < nj; ++j) {
            const double2 z = sl.at(j, c)[i];
            const double2 h = sw[j];
            w.x -= h.x * z.x - h.y * z.y;
            w.y -= h.x * z.y + h.y * z.x;
        }
        y[i] = w;
        acc = fma(w.x, w.x, acc);
        acc = fma(w.y, w.y, acc);
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s;
}

// Several outputs from one pass over the Krylov slots of column c:
// out_o = sum_j coef[o][j] slot(j, c) for o < nout (nout <= kMaxOut).
constexpr int kMaxOut = 16;
__global__ __launch_bounds__(kThreads) void k_combine_multi(Slots sl, int c, int n, const double2* __restrict__ coef,
                                                            int64_t coef_stride, int nout, double2* __restrict__ out,
                                                            int64_t out_col, int64_t D) {
    extern __shared__ double2 sc2[];
    for (int t = threadIdx.x; t < n * nout; t += blockDim.x) sc2[t] = coef[(t / n) * coef_stride + t % n];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re[kMaxOut], im[kMaxOut];
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o) re[o] = im[o] = 0.0;
        for (int j = 0; j < n; ++j) {
            const double2 z = sl.at(j, c)[i];
#pragma unroll
            for (int o = 0; o < kMaxOut; ++o)
                if (o < nout) {
                    const double2 h = sc2[o * n + j];
                    re[o] = fma(h.x, z.x, fma(-h.y, z.y, re[o]));
                    im[o] = fma(h.x, z.y, fma(h.y, z.x, im[o]));
                }
        }
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o)
            if (o < nout) out[o * out_col + i] = make_double2(re[o], im[o]);
    }
}

// out_c = sum_j coef_j slot(j, c)   (coef complex, already including s_j);
// out may alias slot 0 (each element is read before it is written).
__global__ __launch_bounds__(kThreads) void k_combine(Slots sl, int n, const double2* __restrict__ coef,
                                                      int64_t coef_col, double2* __restrict__ out,
                                                      int64_t out_col, int64_t D) {
    extern __shared__ double2 sc[];
    const int c = blockIdx.y;
    for (int j = threadIdx.x; j < n; j += blockDim.x) sc[j] = coef[c * coef_col + j];
    __syncthreads();
    double2* o = out + c * out_col;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; ++j) {
            const double2 z = ld_once(sl.at(j, c) + i);
            const double2 h = sc[j];
            re = fma(h.x, z.x, fma(-h.y, z.y, re));
            im = fma(h.x, z.y, fma(h.y, z.x, im));
        }
        o[i] = make_double2(re, im);
    }
}

__global__ __launch_bounds__(kThreads) void k_scale(double2* __restrict__ x, int64_t D,
                                                    const double* __restrict__ fac) {
    const double f = *fac;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 z = x[i];
        x[i] = make_double2(z.x * f, z.y * f);
    }
}

// ---------------------------------------------------------------------------
// finalisers (one block per column): fixed-order sums of block partials
// ---------------------------------------------------------------------------
__device__ double fixed_sum(const double* p, int n, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += p[i];
    return block_sum(acc, sh);   // thread 0
}

enum FinMode { FIN_INIT = 0, FIN_A = 1, FIN_B = 2 };

__device__ __forceinline__ void fin_body(int mode, int k, double v, double* sc, double tol);

__global__ void k_fin(int mode, int k, const double* __restrict__ part, int nper,
                      double* __restrict__ scal, double tol) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.x;
    double v = fixed_sum(part + (int64_t)c * nper, nper, sh);
    if (threadIdx.x != 0) return;
    fin_body(mode, k, v, scal + (int64_t)c * kScalStride, tol);
}

// finaliser of a grouped launch: column c's partials (rows = 1: one per H.v
// row, else one per streaming block)
__global__ void k_fin_groups(int mode, int k, const GroupCol* __restrict__ cols, int rows,
                             double* __restrict__ scal, double tol) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.x;
    const GroupCol C = cols[c];
    double v = fixed_sum(C.part, rows ? C.nrow : C.nb, sh);
    if (threadIdx.x != 0) return;
    fin_body(mode, k, v, scal + (int64_t)c * kScalStride, tol);
}

__device__ __forceinline__ void fin_body(int mode, int k, double v, double* sc, double tol) {
    if (mode == FIN_INIT) {
        double b0 = sqrt(v);
        sc[kOffBeta0] = b0;
        sc[kOffS] = b0 > 0.0 ? 1.0 / b0 : 0.0;
        sc[kOffB] = 0.0;
        sc[kOffSmax] = 0.0;
    } else if (mode == FIN_A) {
        sc[kOffA + k] = sc[kOffS + k] != 0.0 ? v : 0.0;
    } else {
        double smax = fmax(sc[kOffSmax], fmax(fabs(sc[kOffA + k]), sc[kOffB + k]));
        sc[kOffSmax] = smax;
        double nb = sqrt(v);
        if (sc[kOffS + k] == 0.0 || !(nb > tol * smax)) {
            sc[kOffB + k + 1] = 0.0;
            sc[kOffS + k + 1] = 0.0;
        } else {
            sc[kOffB + k + 1] = nb;
            sc[kOffS + k + 1] = 1.0 / nb;
        }
    }
}

// drift[c] = max(drift[c], | sqrt(sum of column c's partials) / beta0 - 1 |)
__global__ void k_drift_fin(const double* __restrict__ part, int nper, const double* __restrict__ scal,
                            double* __restrict__ drift) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.x;
    const double v = fixed_sum(part + (int64_t)c * nper, nper, sh);
    if (threadIdx.x != 0) return;
    const double b0 = scal[(int64_t)c * kScalStride + kOffBeta0];
    const double d = b0 > 0.0 ? fabs(sqrt(v) / b0 - 1.0) : 0.0;
    drift[c] = fmax(drift[c], d);
}

// sum the multi-dot partials: hvec[c][j] (complex) for j < nj
__global__ void k_fin_h(const double* __restrict__ part, int nj, int nper, double2* __restrict__ hvec) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.x;
    for (int j = 0; j < nj; ++j) {
        double re = fixed_sum(part + (((int64_t)c * nj + j) * 2 + 0) * nper, nper, sh);
        __syncthreads();
        double im = fixed_sum(part + (((int64_t)c * nj + j) * 2 + 1) * nper, nper, sh);
        __syncthreads();
        if (threadIdx.x == 0) hvec[(int64_t)c * nj + j] = make_double2(re, im);
    }
}

// ---------------------------------------------------------------------------
// tridiagonal eigen-decomposition and exponential, one block per column:
// one wavefront (NT = 64) for m <= 64, two (NT = 128) up to kMaxKrylov
// ---------------------------------------------------------------------------
// Implicit QL iteration with Wilkinson shifts for the symmetric tridiagonal
// T (diagonal a_0..a_{m-1}, off-diagonal b_1..b_{m-1}).  Thread 0 chases the
// bulge and records the plane rotations of a sweep; every thread then applies
// them to its own row of the eigenvector matrix Q held in LDS (dynamic,
// m x (m+1) doubles).  Finally
//   coef_k = beta0 * sum_j Q[k][j] f(lambda_j) Q[0][j] * s_k,
// f = exp(-i lambda dt), exp(+i lambda dt) or exp(-(lambda - shift) dt).
// Up to kMaxReq coefficient requests per launch: request r evaluates column
// col[r] at time t[r] with direction dir[r]; its coefficients (including the
// scales s_k) go to coef_out + r * coef_stride (complex).
constexpr int kMaxReq = 64;
struct CoefReq {
    int n;
    int col[kMaxReq];
    int dir[kMaxReq];
    double t[kMaxReq];
};

template <int NT>
__global__ __launch_bounds__(NT) void k_tridiag_exp(const double* __restrict__ scal, int m, CoefReq req,
                                                    double shift, double2* __restrict__ coef_out,
                                                    int coef_stride) {
    extern __shared__ double Qd[];   // Q[i][j] = Qd[i * (m + 1) + j]
    __shared__ double d[kMaxKrylov], e[kMaxKrylov];
    __shared__ double rc[kMaxKrylov], rs[kMaxKrylov];
    __shared__ double xr[NT > 64 ? NT : 1], xi[NT > 64 ? NT : 1];   // neighbour exchange (NT > 64)
    __shared__ double s_red[2][2];
    __shared__ int s_mm, s_lo;
    const int ld = m + 1;
    const int r = blockIdx.x;
    const int c = req.col[r];
    const double dt = req.t[r];
    const int direction = req.dir[r];
    const int lane = threadIdx.x;
    const double* sc = scal + (int64_t)c * kScalStride;
    double2* co = coef_out + (int64_t)r * coef_stride;
    const double beta0 = sc[kOffBeta0];

    // ---- moderate ||T dt||: exp(A) e_1 by n_sub Taylor substeps of exp(A/n_sub),
    // with A = -i (T - sigma) dt, +i (T - sigma) dt or -(T - sigma) dt and
    // the scalar factor of the centre sigma of the Gershgorin interval applied
    // at the end.  Thread r holds row r; the tridiagonal product takes the
    // neighbouring rows by lane shuffles (one wavefront) or through LDS (two
    // wavefronts).  Each substep has x = ||A||/n_sub <= 1 and
    // K terms with x^(K+1)/(K+1)! e^x < 1e-17.  Large ||T dt|| (few long
    // steps) takes the eigen-decomposition below instead.
    {
        const double a0 = lane < m ? sc[kOffA + lane] : 0.0;
        const double br = (lane >= 1 && lane < m) ? sc[kOffB + lane] : 0.0;          // couples r-1, r
        const double bn = (lane + 1 < m) ? sc[kOffB + lane + 1] : 0.0;              // couples r, r+1
        double glo = lane < m ? a0 - fabs(br) - fabs(bn) : DBL_MAX;
        double ghi = lane < m ? a0 + fabs(br) + fabs(bn) : -DBL_MAX;
        for (int off = 32; off > 0; off >>= 1) {
            glo = fmin(glo, __shfl_xor(glo, off, 64));
            ghi = fmax(ghi, __shfl_xor(ghi, off, 64));
        }
        if (NT > 64) {
            if ((lane & 63) == 0) {
                s_red[lane >> 6][0] = glo;
                s_red[lane >> 6][1] = ghi;
            }
            __syncthreads();
            glo = fmin(s_red[0][0], s_red[1][0]);
            ghi = fmax(s_red[0][1], s_red[1][1]);
        }
        const double sigma = 0.5 * (glo + ghi);
        const double x = 0.5 * (ghi - glo) * fabs(dt);
        if (x <= 64.0) {
            const int n_sub = x <= 1.0 ? 1 : (int)ceil(x);
            const double xs = x / n_sub;
            int K = 1;
            {
                double term = xs, fact = 1.0;
                const double ex = exp(xs);
                while (K < 40) {
                    fact *= (double)(K + 1);
                    term *= xs;
                    if (term / fact * ex < 1e-17) break;
                    ++K;
                }
            }
            const double ar = a0 - sigma;
            const double h = dt / n_sub;
            double cr = lane == 0 ? 1.0 : 0.0, ci = 0.0;   // current state
            for (int sub = 0; sub < n_sub; ++sub) {
                double vr = cr, vi = ci;                     // running term
                for (int k = 1; k <= K; ++k) {
                    double pr, pi, nr, ni;
                    if (NT == 64) {
                        pr = __shfl_up(vr, 1, 64);
                        pi = __shfl_up(vi, 1, 64);
                        nr = __shfl_down(vr, 1, 64);
                        ni = __shfl_down(vi, 1, 64);
                    } else {
                        xr[lane] = vr;
                        xi[lane] = vi;
                        __syncthreads();
                        pr = lane >= 1 ? xr[lane - 1] : 0.0;
                        pi = lane >= 1 ? xi[lane - 1] : 0.0;
                        nr = lane + 1 < NT ? xr[lane + 1] : 0.0;
                        ni = lane + 1 < NT ? xi[lane + 1] : 0.0;
                        __syncthreads();
                    }
                    const double wr = ar * vr + (lane >= 1 ? br * pr : 0.0) + (lane + 1 < m ? bn * nr : 0.0);
                    const double wi = ar * vi + (lane >= 1 ? br * pi : 0.0) + (lane + 1 < m ? bn * ni : 0.0);
                    const double f = h / (double)k;
                    if (direction == 0) {        // -(T - sigma) h
                        vr = -f * wr;
                        vi = -f * wi;
                    } else if (direction < 0) {  // -i (T - sigma) h
                        vr = f * wi;
                        vi = -f * wr;
                    } else {                     // +i (T - sigma) h
                        vr = -f * wi;
                        vi = f * wr;
                    }
                    if (lane >= m) vr = vi = 0.0;
                    cr += vr;
                    ci += vi;
                }
            }
            // scalar factor of the centre: exp(-i sigma dt), exp(+i sigma dt) or exp(-(sigma - shift) dt)
            double fr, fi;
            if (direction == 0) {
                fr = exp(-(sigma - shift) * dt);
                fi = 0.0;
            } else {
                double sn, cs;
                sincos(sigma * dt, &sn, &cs);
                fr = cs;
                fi = direction < 0 ? -sn : sn;
            }
            if (lane < m) {
                const double g = beta0 * sc[kOffS + lane];
                co[lane] = make_double2((cr * fr - ci * fi) * g, (cr * fi + ci * fr) * g);
            }
            return;
        }
    }

    if (lane < m) {
        d[lane] = sc[kOffA + lane];
        e[lane] = lane + 1 < m ? sc[kOffB + lane + 1] : 0.0;
        for (int j = 0; j < m; ++j) Qd[lane * ld + j] = (j == lane) ? 1.0 : 0.0;
    }
    __syncthreads();

    for (int l = 0; l < m; ++l) {
        for (int iter = 0; iter < 64; ++iter) {
            if (lane == 0) {
                int mm = l;
                for (; mm < m - 1; ++mm) {
                    const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                    if (fabs(e[mm]) <= DBL_EPSILON * dd) break;
                }
                s_mm = mm;
                if (mm != l) {
                    double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                    double r = hypot(g, 1.0);
                    g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
                    double s = 1.0, cc = 1.0, p = 0.0;
                    int i = mm - 1;
                    bool deflated = false;
                    for (; i >= l; --i) {
                        const double f = s * e[i];
                        const double b = cc * e[i];
                        r = hypot(f, g);
                        e[i + 1] = r;
                        if (r == 0.0) {
                            d[i + 1] -= p;
                            e[mm] = 0.0;
                            deflated = true;
                            break;
                        }
                        s = f / r;
                        cc = g / r;
                        g = d[i + 1] - p;
                        r = (d[i] - g) * s + 2.0 * cc * b;
                        p = s * r;
                        d[i + 1] = g + p;
                        g = cc * r - b;
                        rc[i] = cc;
                        rs[i] = s;
                    }
                    if (!deflated) {
                        d[l] -= p;
                        e[l] = g;
                        e[mm] = 0.0;
                        s_lo = l;
                    } else {
                        s_lo = i + 1;
                    }
                }
            }
            __syncthreads();
            const int mm = s_mm;
            if (mm == l) break;
            if (lane < m) {
                double* Qr = Qd + lane * ld;
                for (int i = mm - 1; i >= s_lo; --i) {
                    const double f = Qr[i + 1];
                    const double q = Qr[i];
                    Qr[i + 1] = rs[i] * q + rc[i] * f;
                    Qr[i] = rc[i] * q - rs[i] * f;
                }
            }
            __syncthreads();
        }
    }

    if (lane < m) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < m; ++j) {
            double fr, fi;
            if (direction == 0) {
                fr = exp(-(d[j] - shift) * dt);
                fi = 0.0;
            } else {
                double sn, cs;
                sincos(d[j] * dt, &sn, &cs);
                fr = cs;
                fi = direction < 0 ? -sn : sn;
            }
            const double w = Qd[lane * ld + j] * Qd[j];
            re = fma(w, fr, re);
            im = fma(w, fi, im);
        }
        const double f = beta0 * sc[kOffS + lane];
        co[lane] = make_double2(re * f, im * f);
    }
}

// ---------------------------------------------------------------------------
// ground state of T_n: lowest eigenvalue by multisection of Sturm counts
// (64 lanes), eigenvector by inverse iteration on lane 0.
// ---------------------------------------------------------------------------
__device__ int sturm_count(const double* a, const double* b2, int n, double x) {
    // number of eigenvalues of T below x (LDL^T pivots of T - x I)
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < n; ++i) {
        if (q == 0.0) q = DBL_MIN;   // perturb an exact zero pivot
        q = a[i] - x - b2[i] / q;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// gs arrays: a[n], b[n+1] (b[0] = 0, b[k] couples k-1, k), scratch >= 6 n doubles
// out: res[0] = E0, res[1] = residual, res[2] = n_eff, res[3] = broken flag;
//      y[0..n_eff-1] eigenvector (unit norm, largest-magnitude entry positive)
__global__ __launch_bounds__(64) void k_gs_eig(const double* __restrict__ a, const double* __restrict__ b,
                                               int n, double* __restrict__ scratch,
                                               double* __restrict__ y, double* __restrict__ res) {
    __shared__ double s_lo, s_hi;
    __shared__ int s_n;
    __shared__ int s_cnt[64];
    const int lane = threadIdx.x;
    if (lane == 0) {
        int ne = n;
        for (int i = 1; i < n; ++i)
            if (b[i] == 0.0) {
                ne = i;
                break;
            }
        s_n = ne;
        double lo = DBL_MAX, hi = -DBL_MAX;
        double* b2 = scratch;
        for (int i = 0; i < ne; ++i) {
            b2[i] = i > 0 ? b[i] * b[i] : 0.0;
            const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < ne ? fabs(b[i + 1]) : 0.0);
            lo = fmin(lo, a[i] - r);
            hi = fmax(hi, a[i] + r);
        }
        s_lo = lo - 1e-300;
        s_hi = hi + 1e-300;
    }
    __syncthreads();
    const int ne = s_n;
    const double* b2 = scratch;
    for (int round = 0; round < 40; ++round) {
        const double lo = s_lo, hi = s_hi;
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) || hi - lo <= DBL_MIN) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        s_cnt[lane] = sturm_count(a, b2, ne, x);
        __syncthreads();
        if (lane == 0) {
            int l = 0;
            while (l < 64 && s_cnt[l] < 1) ++l;
            const double nlo = l == 0 ? lo : lo + (hi - lo) * (double)l / 65.0;
            const double nhi = l == 64 ? hi : lo + (hi - lo) * (double)(l + 1) / 65.0;
            s_lo = nlo;
            s_hi = fmin(nhi, hi);
        }
        __syncthreads();
    }
    if (lane != 0) return;
    const double lam = 0.5 * (s_lo + s_hi);
    // inverse iteration: (T - lam I) z = y, LU with partial pivoting
    double* dl = scratch + ne;        // sub-diagonal multipliers
    double* du = dl + ne;             // U diagonal
    double* u1 = du + ne;             // U first super-diagonal
    double* u2 = u1 + ne;             // U second super-diagonal (fill-in)
    int* piv = reinterpret_cast<int*>(u2 + ne);
    double tnorm = 0.0;
    for (int i = 0; i < ne; ++i) tnorm = fmax(tnorm, fabs(a[i]) + (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < ne ? fabs(b[i + 1]) : 0.0));
    const double tiny = DBL_EPSILON * fmax(tnorm, DBL_MIN);
    // factor
    for (int i = 0; i < ne; ++i) {
        du[i] = a[i] - lam;
        u1[i] = i + 1 < ne ? b[i + 1] : 0.0;
        u2[i] = 0.0;
    }
    for (int i = 0; i < ne - 1; ++i) {
        const double sub = b[i + 1];
        if (fabs(du[i]) >= fabs(sub)) {
            piv[i] = 0;
            const double piv_v = du[i] != 0.0 ? du[i] : tiny;
            du[i] = piv_v;
            const double f = sub / piv_v;
            dl[i] = f;
            du[i + 1] -= f * u1[i];
        } else {
            piv[i] = 1;
            const double f = du[i] / sub;
            dl[i] = f;
            // swap rows i and i+1
            const double r_d = sub, r_u1 = du[i + 1], r_u2 = i + 1 < ne - 1 ? u1[i + 1] : 0.0;
            const double o_u1 = u1[i];
            du[i] = r_d;
            u1[i] = r_u1;
            u2[i] = r_u2;
            du[i + 1] = o_u1 - f * r_u1;
            if (i + 1 < ne - 1) u1[i + 1] = -f * r_u2;
        }
    }
    if (du[ne - 1] == 0.0) du[ne - 1] = tiny;
    for (int i = 0; i < ne; ++i) y[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
        // forward (L)
        for (int i = 0; i < ne - 1; ++i) {
            if (piv[i]) {
                const double t = y[i];
                y[i] = y[i + 1];
                y[i + 1] = t - dl[i] * y[i];
            } else {
                y[i + 1] -= dl[i] * y[i];
            }
        }
        // backward (U)
        for (int i = ne - 1; i >= 0; --i) {
            double s = y[i];
            if (i + 1 < ne) s -= u1[i] * y[i + 1];
            if (i + 2 < ne) s -= u2[i] * y[i + 2];
            y[i] = s / du[i];
        }
        double nrm = 0.0, big = 0.0;
        int ib = 0;
        for (int i = 0; i < ne; ++i) {
            nrm = fma(y[i], y[i], nrm);
            if (fabs(y[i]) > big) {
                big = fabs(y[i]);
                ib = i;
            }
        }
        nrm = sqrt(nrm);
        const double f = (y[ib] < 0.0 ? -1.0 : 1.0) / nrm;
        for (int i = 0; i < ne; ++i) y[i] *= f;
    }
    for (int i = ne; i < n; ++i) y[i] = 0.0;
    res[0] = lam;
    res[1] = (ne < n) ? 0.0 : fabs(b[n]) * fabs(y[ne - 1]);
    res[2] = (double)ne;
    res[3] = ne < n ? 1.0 : (b[n] == 0.0 ? 1.0 : 0.0);
}

// GS recursion scalars live in plain arrays: a[k], b[k], s[k]
__global__ void k_gs_fin(int mode, int k, const double* __restrict__ part, int nper,
                         double* __restrict__ a, double* __restrict__ b, double* __restrict__ s) {
    __shared__ double sh[kThreads / 64];
    double v = fixed_sum(part, nper, sh);
    if (threadIdx.x != 0) return;
    if (mode == FIN_INIT) {
        double n0 = sqrt(v);
        s[0] = n0 > 0.0 ? 1.0 / n0 : 0.0;
        b[0] = 0.0;
    } else if (mode == FIN_A) {
        a[k] = s[k] != 0.0 ? v : 0.0;
    } else {
        double nb = sqrt(v);
        if (s[k] == 0.0 || nb == 0.0) {
            b[k + 1] = 0.0;
            s[k + 1] = 0.0;
        } else {
            b[k + 1] = nb;
            s[k + 1] = 1.0 / nb;
        }
    }
}

__global__ void k_gs_coef(const double* __restrict__ y, const double* __restrict__ s, int n,
                          double2* __restrict__ coef) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) coef[j] = make_double2(y[j] * s[j], 0.0);
}

__global__ void k_inv_sqrt(const double* __restrict__ part, int nper, double* __restrict__ out) {
    __shared__ double sh[kThreads / 64];
    double v = fixed_sum(part, nper, sh);
    if (threadIdx.x == 0) *out = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
}

// block dots: out[l * nr + r] = <L_l | R_r>
__global__ __launch_bounds__(kThreads) void k_dots(const double2* __restrict__ Lv, int64_t l_col, int nl,
                                                   const double2* __restrict__ Rv, int64_t r_col,
                                                   const double2* const* __restrict__ Rptr, int64_t D,
                                                   double* __restrict__ part) {
    __shared__ double sh[kThreads / 64][2 * kDotChunk];
    const int r = blockIdx.y;
    const int l0 = blockIdx.z * kDotChunk;
    const int nloc = nl - l0 < kDotChunk ? nl - l0 : kDotChunk;
    const double2* R = Rptr ? Rptr[r] : Rv + r * r_col;
    double ar[kDotChunk], ai[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) ar[q] = ai[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 w = R[i];
#pragma unroll
        for (int q = 0; q < kDotChunk; ++q) {
            if (q < nloc) {
                const double2 z = Lv[(l0 + q) * l_col + i];
                ar[q] = fma(z.x, w.x, fma(z.y, w.y, ar[q]));
                ai[q] = fma(z.x, w.y, fma(-z.y, w.x, ai[q]));
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
        double x = wave_sum(ar[q]);
        double y = wave_sum(ai[q]);
        if (lane == 0) {
            sh[wv][2 * q] = x;
            sh[wv][2 * q + 1] = y;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nloc) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w][threadIdx.x];
        const int l = l0 + (threadIdx.x >> 1);
        part[(((int64_t)l * gridDim.y + r) * 2 + (threadIdx.x & 1)) * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void k_dots_fin(const double* __restrict__ part, int nper, int nr, int64_t out_ld,
                           double2* __restrict__ out) {
    __shared__ double sh[kThreads / 64];
    const int idx = blockIdx.x;   // l * nr + r
    double re = fixed_sum(part + ((int64_t)idx * 2 + 0) * nper, nper, sh);
    __syncthreads();
    double im = fixed_sum(part + ((int64_t)idx * 2 + 1) * nper, nper, sh);
    if (threadIdx.x == 0) out[(int64_t)(idx / nr) * out_ld + idx % nr] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
void launch_fin(kgf_ctx* ctx, int mode, int k, const double* part, int nper, double* scal, int ncol,
                double tol) {
    Prof pr(ctx, "fin");
    hipLaunchKernelGGL(k_fin, dim3(ncol), dim3(kThreads), 0, ctx->stream, mode, k, part, nper, scal, tol);
    check_launch("k_fin");
}

// Gram-Schmidt against slots 0..nj-1 (coefficients in hvec), `passes` times.
// Leaves ||y||^2 partials of the last pass in part (nper = red_blocks(D)).
void reorthogonalise(kgf_ctx* ctx, const Slots& sl, int ky, int nj, int ncol, int64_t D, int passes,
                     const double* scal, const double* gs_s, double* part, double* part_big,
                     double2* hvec) {
    const int NB = red_blocks(D);
    const int nchunk = (nj + kDotChunk - 1) / kDotChunk;
    for (int p = 0; p < passes; ++p) {
        {
            Prof pr(ctx, "reorth_dot");
            hipLaunchKernelGGL(k_multidot, dim3(NB, ncol, nchunk), dim3(kThreads), 0, ctx->stream, sl,
                               ky, nj, scal, gs_s, D, part_big);
            check_launch("k_multidot");
        }
        {
            Prof pr(ctx, "fin");
            hipLaunchKernelGGL(k_fin_h, dim3(ncol), dim3(kThreads), 0, ctx->stream, part_big, nj, NB, hvec);
            check_launch("k_fin_h");
        }
        {
            Prof pr(ctx, "reorth_axpy");
            hipLaunchKernelGGL(k_multiaxpy, dim3(NB, ncol), dim3(kThreads), sizeof(double2) * nj,
                               ctx->stream, sl, ky, nj, scal, gs_s, hvec, D, part);
            check_launch("k_multiaxpy");
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// short-iterative-Lanczos propagation
// ---------------------------------------------------------------------------
void sil_reserve(kgf_ctx* ctx, const kgf_sector* sec, int ncol, int m, int reorth) {
    const int64_t D = sec->dim();
    const size_t xbytes = sizeof(double2) * (size_t)m * ncol * D;
    auto& xs = ctx->ws["sil_X"];
    if (!xs || xs->bytes < xbytes) {
        if (xs) {   // free the smaller buffer first so that the new one fits
            sync(ctx);
            xs.reset();
        }
        ensure_device_fits(xbytes, "SIL Krylov basis");
        workspace(ctx, "sil_X", xbytes);
    }
    const int NB = red_blocks(D);
    const int HB = hv_part_capacity(ctx, sec);   // partials of either H.v pass
    const int nper_max = NB > HB ? NB : HB;
    workspace(ctx, "sil_scal", sizeof(double) * kScalStride * ncol);
    workspace(ctx, "sil_part", sizeof(double) * (size_t)nper_max * ncol);
    if (reorth > 0) {
        workspace(ctx, "sil_partbig", sizeof(double) * (size_t)NB * ncol * (m + 1) * 2);
        workspace(ctx, "sil_hvec", sizeof(double2) * (size_t)ncol * (m + 1));
    }
}

// A-posteriori estimate of one SIL step's error.  The Krylov state
// u(t) = beta0 V_m f(t T_m) e_1 leaves the residual r(t) = A u - u' =
// beta0 b_m [f(t T_m) e_1]_{m-1} v_m (A = -+iH, or -(H - shift)), and the
// error of the step is int_0^dt e^{(dt - t) A} r(t) dt, so
//     err <= beta0 b_m int_0^dt |[f(t T_m) e_1]_{m-1}| dt
// (with the norm of e^{(dt - t) A} at most 1: real time, or imaginary time
// with the shift at or below the spectrum).  The integral is taken with a
// kErrNodes-point Gauss-Legendre rule on [0, dt]; the coefficients at the
// nodes are coef_k = beta0 u_k s_k, so beta0 |u_{m-1}| = |coef_{m-1}| / s_{m-1}.
// err[c] keeps the largest value over the steps.
constexpr int kErrNodes = 16;
struct GlRule {
    double x[kErrNodes];   // nodes on [0, 1]
    double w[kErrNodes];   // weights, summing to 1
};

// Gauss-Legendre rule on [0, 1]: the roots of P_n by Newton's method from
// the Chebyshev-like first guesses, weights 2 / ((1 - z^2) P_n'(z)^2) halved.
static GlRule make_gl_rule() {
    GlRule g;
    const int n = kErrNodes;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        g.x[i] = 0.5 * (1.0 - z);
        g.w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return g;
}

static const GlRule& gl_rule() {
    static const GlRule g = make_gl_rule();
    return g;
}

__global__ void k_err_est(const double* __restrict__ scal, int m, int ncol, const double2* __restrict__ nodec,
                          GlRule g, double dt, double* __restrict__ err) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const double* sc = scal + (int64_t)c * kScalStride;
    const double s = sc[kOffS + m - 1];
    double e = 0.0;
    if (s != 0.0) {
        double acc = 0.0;
        for (int i = 0; i < kErrNodes; ++i) {
            const double2 cf = nodec[((int64_t)c * kErrNodes + i) * m + m - 1];
            acc += g.w[i] * hypot(cf.x, cf.y);
        }
        e = fabs(dt) * sc[kOffB + m] * acc / s;
    }
    err[c] = fmax(err[c], e);
}

__global__ void k_fill_zero(double* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Device memory of one batched SIL step: the Krylov slots 1..m (slot 0 is
// the state itself), the per-column scalars, the reduction partials and,
// with reorthogonalisation, the Gram-Schmidt partials and coefficients.
struct SilWork {
    double2* X;
    double* scal;
    double* part;
    double* part_big;
    double2* hvec;
    double* err;      // per-column running maximum of the step error estimate, or null
    double* drift;    // per-column running maximum of | ||psi_after|| / ||psi_before|| - 1 |, or null
    double2* errc;    // [ncol][kErrNodes][m] coefficients at the estimate's quadrature nodes (with err)
};

// Byte layout of a SilWork carved from one buffer (each piece 256-aligned).
struct SilLayout {
    size_t x, scal, part, part_big, hvec, err, errc, total;
};
static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
static SilLayout sil_layout(kgf_ctx* ctx, const kgf_sector* sec, int ncol, int m, int reorth) {
    const int64_t D = sec->dim();
    const int NB = red_blocks(D);
    const int HB = hv_part_capacity(ctx, sec);   // partials of either H.v pass
    const int nper_max = NB > HB ? NB : HB;
    SilLayout l;
    l.x = 0;
    l.scal = l.x + align256(sizeof(double2) * (size_t)m * ncol * D);
    l.part = l.scal + align256(sizeof(double) * kScalStride * ncol);
    l.part_big = l.part + align256(sizeof(double) * (size_t)nper_max * ncol);
    l.hvec = l.part_big + (reorth > 0 ? align256(sizeof(double) * (size_t)NB * ncol * (m + 1) * 2) : 0);
    l.err = l.hvec + (reorth > 0 ? align256(sizeof(double2) * (size_t)ncol * (m + 1)) : 0);
    l.errc = l.err + align256(sizeof(double) * (size_t)ncol);
    l.total = l.errc + align256(sizeof(double2) * (size_t)ncol * kErrNodes * m);
    return l;
}

// Lanczos bases of ncol columns psi_c = psi + c * ld (slot 0 = psi itself)
// in the memory of w; the scalars are left in w.scal.
static void sil_build_w(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                        const SilOpts& o, const SilWork& w) {
    const int64_t D = sec->dim();
    const int m = o.m;
    double2* X = w.X;
    double* scal = w.scal;
    const int NB = red_blocks(D);
    const int HB = hv_lanczos_blocks(ctx, sec);
    double* part = w.part;
    double* part_big = w.part_big;
    double2* hvec = w.hvec;
    Slots sl{psi, ld, X, (int64_t)ncol * D, D};
    {
        Prof pr(ctx, "norm", 16.0 * D * ncol);
        hipLaunchKernelGGL(k_norm2, dim3(NB, ncol), dim3(kThreads), 0, ctx->stream, psi, ld, D, part);
        check_launch("k_norm2");
    }
    launch_fin(ctx, FIN_INIT, 0, part, NB, scal, ncol, 0.0);
    int UB = 0;   // pass-2 partials of a fused step
    const int RB = (o.reorth == 0 && ctx->hv_fuse) ? hv_lanczos_rows_blocks(ctx, model, sec, ncol, &UB) : 0;
    if (RB > 0) {
        // two-pass H.v: the update of step k - 1 rides in the row pass of step k
        for (int k = 0; k < m; ++k) {
            LanczosRowsArgs r;
            r.x = sl.at(k, 0);
            r.x_col = k == 0 ? ld : D;
            r.z = sl.at(k + 1, 0);
            r.z_col = D;
            r.xp = k > 0 ? sl.at(k - 1, 0) : nullptr;
            r.xp_col = k - 1 == 0 ? ld : D;
            r.fa = scal + kOffA + (k > 0 ? k - 1 : 0);
            r.fs = scal + kOffS + (k > 0 ? k - 1 : 0);
            r.stride = kScalStride;
            r.part = part;
            hv_lanczos_rows(ctx, model, sec, ncol, r);
            if (k > 0) launch_fin(ctx, FIN_B, k - 1, part, RB, scal, ncol, o.breakdown_tol);
            LanczosHvArgs a;
            a.x = sl.at(k, 0);
            a.x_col = k == 0 ? ld : D;
            a.xp = k > 0 ? sl.at(k - 1, 0) : nullptr;
            a.xp_col = k - 1 == 0 ? ld : D;
            a.y = sl.at(k + 1, 0);
            a.y_col = D;
            a.s_k = scal + kOffS + k;
            a.b_k = scal + kOffB + k;
            a.s_km1 = scal + kOffS + (k > 0 ? k - 1 : 0);
            a.stride = kScalStride;
            a.part = part;
            hv_lanczos_up(ctx, model, sec, ncol, a);
            launch_fin(ctx, FIN_A, k, part, UB, scal, ncol, 0.0);
        }
        if (w.err) {   // b_m for the error estimate
            {
                Prof pr(ctx, "lanczos_update", 48.0 * D * ncol);
                hipLaunchKernelGGL(k_update, dim3(NB, ncol), dim3(kThreads), 0, ctx->stream, sl, m - 1,
                                   scal + kOffA + m - 1, scal + kOffS + m - 1, kScalStride, D, part);
                check_launch("k_update");
            }
            launch_fin(ctx, FIN_B, m - 1, part, NB, scal, ncol, o.breakdown_tol);
        }
        return;
    }
    for (int k = 0; k < m; ++k) {
        LanczosHvArgs a;
        a.x = sl.at(k, 0);
        a.x_col = k == 0 ? ld : D;
        a.xp = k > 0 ? sl.at(k - 1, 0) : nullptr;
        a.xp_col = k - 1 == 0 ? ld : D;
        a.y = sl.at(k + 1, 0);
        a.y_col = D;
        a.s_k = scal + kOffS + k;
        a.b_k = scal + kOffB + k;
        a.s_km1 = scal + kOffS + (k > 0 ? k - 1 : 0);
        a.stride = kScalStride;
        a.part = part;
        hv_lanczos(ctx, model, sec, ncol, a);
        launch_fin(ctx, FIN_A, k, part, HB, scal, ncol, 0.0);
        if (k == m - 1 && !w.err) break;   // b_m only for the error estimate
        {
            Prof pr(ctx, "lanczos_update", 48.0 * D * ncol);
            hipLaunchKernelGGL(k_update, dim3(NB, ncol), dim3(kThreads), 0, ctx->stream, sl, k,
                               scal + kOffA + k, scal + kOffS + k, kScalStride, D, part);
            check_launch("k_update");
        }
        if (o.reorth > 0 && k < m - 1)
            reorthogonalise(ctx, sl, k + 1, k + 1, ncol, D, o.reorth, scal, nullptr, part, part_big, hvec);
        launch_fin(ctx, FIN_B, k, part, NB, scal, ncol, o.breakdown_tol);
    }
}

// The SIL buffers in the context's workspaces (sil_reserve first).
static SilWork sil_work_ws(kgf_ctx* ctx, const kgf_sector* sec, int ncol, const SilOpts& o) {
    const int64_t D = sec->dim();
    const int NB = red_blocks(D);
    const int HB = hv_part_capacity(ctx, sec);   // partials of either H.v pass
    const int nper_max = NB > HB ? NB : HB;
    SilWork w;
    w.X = static_cast<double2*>(workspace(ctx, "sil_X", sizeof(double2) * (size_t)o.m * ncol * D));
    w.scal = static_cast<double*>(workspace(ctx, "sil_scal", sizeof(double) * kScalStride * ncol));
    w.part = static_cast<double*>(workspace(ctx, "sil_part", sizeof(double) * (size_t)nper_max * ncol));
    w.part_big = nullptr;
    w.hvec = nullptr;
    if (o.reorth > 0) {
        w.part_big = static_cast<double*>(
            workspace(ctx, "sil_partbig", sizeof(double) * (size_t)NB * ncol * (o.m + 1) * 2));
        w.hvec = static_cast<double2*>(workspace(ctx, "sil_hvec", sizeof(double2) * (size_t)ncol * (o.m + 1)));
    }
    w.err = nullptr;
    w.errc = nullptr;
    w.drift = nullptr;
    return w;
}

// Lanczos bases of ncol columns psi_c = psi + c * ld (slot 0 = psi itself);
// leaves the scalars in "sil_scal" and slots 1..m in "sil_X".
void sil_build(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
               const SilOpts& o) {
    KGF_REQUIRE(ncol <= 65535, KGF_EUNSUPPORTED, "SIL: at most 65535 columns per batch");
    hv_prepare(ctx, model, sec, ncol);
    sil_reserve(ctx, sec, ncol, o.m, o.reorth);
    sil_build_w(ctx, model, sec, psi, ncol, ld, o, sil_work_ws(ctx, sec, ncol, o));
}

// exp(T t) e_1 coefficients of up to kMaxReq requests against the scalars at scal
static void launch_coefs(kgf_ctx* ctx, const double* scal, int m, const CoefReq& q, double shift, double2* coef,
                         int coef_stride) {
    Prof pr(ctx, "tridiag_exp");
    const size_t lds = sizeof(double) * (size_t)m * (m + 1);
    if (m <= 64) {
        hipLaunchKernelGGL(k_tridiag_exp<64>, dim3(q.n), dim3(64), lds, ctx->stream, scal, m, q, shift, coef,
                           coef_stride);
    } else {
        static bool opted[64] = {};
        if (!opted[ctx->device & 63]) {
            KGF_HIP(hipFuncSetAttribute((const void*)k_tridiag_exp<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(sizeof(double) * kMaxKrylov * (kMaxKrylov + 1))));
            opted[ctx->device & 63] = true;
        }
        hipLaunchKernelGGL(k_tridiag_exp<128>, dim3(q.n), dim3(128), lds, ctx->stream, scal, m, q, shift, coef,
                           coef_stride);
    }
    check_launch("k_tridiag_exp");
}

// coefficient requests against the bases left by sil_build
void sil_coefs(kgf_ctx* ctx, int m, int nreq, const int* col, const double* t, const int* dir, double shift,
               double2* coef, int coef_stride) {
    const double* scal = static_cast<const double*>(ctx->ws["sil_scal"]->p);
    for (int r0 = 0; r0 < nreq; r0 += kMaxReq) {
        CoefReq q;
        q.n = std::min(kMaxReq, nreq - r0);
        for (int r = 0; r < q.n; ++r) {
            q.col[r] = col[r0 + r];
            q.t[r] = t[r0 + r];
            q.dir[r] = dir[r0 + r];
        }
        launch_coefs(ctx, scal, m, q, shift, coef + (int64_t)r0 * coef_stride, coef_stride);
    }
}

// out + o * out_col = sum_j coef[o][j] v_j(column c) for nout outputs
void sil_combine_multi(kgf_ctx* ctx, const kgf_sector* sec, double2* psi, int64_t ld, int ncol, int m, int c,
                       const double2* coef, int64_t coef_stride, int nout, double2* out, int64_t out_col) {
    const int64_t D = sec->dim();
    double2* X = static_cast<double2*>(ctx->ws["sil_X"]->p);
    Slots sl{psi, ld, X, (int64_t)ncol * D, D};
    const int NB = red_blocks(D);
    for (int o0 = 0; o0 < nout; o0 += kMaxOut) {
        const int no = std::min(kMaxOut, nout - o0);
        Prof pr(ctx, "combine", 16.0 * (m + no) * D);
        hipLaunchKernelGGL(k_combine_multi, dim3(NB), dim3(kThreads), sizeof(double2) * m * no, ctx->stream, sl, c,
                           m, coef + o0 * coef_stride, coef_stride, no, out + o0 * out_col, out_col, D);
        check_launch("k_combine_multi");
    }
}

// One SIL step of every column in the memory of w: build, exp(-+i T dt) e_1
// (column c's coefficients into its scalar block), combination into psi.
static void sil_step_w(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                       const SilOpts& o, const SilWork& w) {
    const int64_t D = sec->dim();
    const int m = o.m;
    sil_build_w(ctx, model, sec, psi, ncol, ld, o, w);
    double2* coef = reinterpret_cast<double2*>(w.scal + kOffCoef);
    for (int r0 = 0; r0 < ncol; r0 += kMaxReq) {
        CoefReq q;
        q.n = std::min(kMaxReq, ncol - r0);
        for (int r = 0; r < q.n; ++r) {
            q.col[r] = r0 + r;
            q.t[r] = o.dt;
            q.dir[r] = o.direction;
        }
        launch_coefs(ctx, w.scal, m, q, o.shift, coef + (int64_t)r0 * (kScalStride / 2), kScalStride / 2);
    }
    if (w.err) {
        const GlRule& g = gl_rule();
        const int nreq = ncol * kErrNodes;
        for (int r0 = 0; r0 < nreq; r0 += kMaxReq) {
            CoefReq q;
            q.n = std::min(kMaxReq, nreq - r0);
            for (int r = 0; r < q.n; ++r) {
                q.col[r] = (r0 + r) / kErrNodes;
                q.t[r] = o.dt * g.x[(r0 + r) % kErrNodes];
                q.dir[r] = o.direction;
            }
            launch_coefs(ctx, w.scal, m, q, o.shift, w.errc + (int64_t)r0 * m, m);
        }
        hipLaunchKernelGGL(k_err_est, dim3((ncol + 63) / 64), dim3(64), 0, ctx->stream, w.scal, m, ncol, w.errc, g,
                           o.dt, w.err);
        check_launch("k_err_est");
    }
    Slots sl{psi, ld, w.X, (int64_t)ncol * D, D};
    const int NB = red_blocks(D);
    Prof pr(ctx, "combine", 16.0 * (m + 1) * D * ncol);
    hipLaunchKernelGGL(k_combine, dim3(NB, ncol), dim3(kThreads), sizeof(double2) * m, ctx->stream, sl, m,
                       reinterpret_cast<const double2*>(coef), (int64_t)(kScalStride / 2), psi, ld, D);
    check_launch("k_combine");
    if (w.drift) {   // norm after the step against beta0, the norm before it
        {
            Prof pn(ctx, "norm", 16.0 * D * ncol);
            hipLaunchKernelGGL(k_norm2, dim3(NB, ncol), dim3(kThreads), 0, ctx->stream, psi, ld, D, w.part);
            check_launch("k_norm2");
        }
        hipLaunchKernelGGL(k_drift_fin, dim3(ncol), dim3(kThreads), 0, ctx->stream, w.part, NB, w.scal, w.drift);
        check_launch("k_drift_fin");
    }
}

// Identity of a batched SIL step for graph replay: everything its launches
// take as arguments (model parameters by version, sector, state buffer,
// batch, options, work buffers).
struct SilStepKey {
    uint64_t model_version;
    int L, n_up, n_dn, ncol;
    const double2* psi;
    int64_t ld;
    int m, reorth, direction;
    double dt, shift, breakdown_tol;
    const void* bufs[5];
};

static std::vector<unsigned char> step_key(HModel model, const kgf_sector* sec, const double2* psi, int ncol,
                                           int64_t ld, const SilOpts& o, const SilWork& w) {
    SilStepKey k;
    std::memset(&k, 0, sizeof(k));
    k.model_version = model.set ? model.set->version : model.m->version;
    k.L = sec->L;
    k.n_up = sec->n_up;
    k.n_dn = sec->n_dn;
    k.ncol = ncol;
    k.psi = psi;
    k.ld = ld;
    k.m = o.m;
    k.reorth = o.reorth;
    k.direction = o.direction;
    k.dt = o.dt;
    k.shift = o.shift;
    k.breakdown_tol = o.breakdown_tol;
    k.bufs[0] = w.X;
    k.bufs[1] = w.scal;
    k.bufs[2] = w.part;
    k.bufs[3] = w.part_big;
    k.bufs[4] = w.hvec;
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&k);
    return std::vector<unsigned char>(b, b + sizeof(k));
}

constexpr size_t kMaxGraphs = 32;

// One SIL step, eager on the first sighting of its key, captured into a
// hipGraph (on a private stream, launched on the context's stream) on the
// second, replayed from then on.  The first eager step also builds any
// tables the launches read, so nothing is allocated or copied synchronously
// during a capture.
static void sil_step_graph(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                           const SilOpts& o, const SilWork& w) {
    std::vector<unsigned char> key = step_key(model, sec, psi, ncol, ld, o, w);
    auto& G = ctx->sil_graphs;
    auto it = std::find_if(G.begin(), G.end(), [&](const kgf_ctx::SilGraph& g) { return g.key == key; });
    if (it == G.end()) {
        sil_step_w(ctx, model, sec, psi, ncol, ld, o, w);
        if (G.size() >= kMaxGraphs) {
            auto old = std::min_element(G.begin(), G.end(), [](const kgf_ctx::SilGraph& a, const kgf_ctx::SilGraph& b) {
                return a.last_use < b.last_use;
            });
            if (old->exec) {
                sync(ctx);
                (void)hipGraphExecDestroy(old->exec);
            }
            G.erase(old);
        }
        kgf_ctx::SilGraph g;
        g.key = std::move(key);
        g.last_use = ++ctx->graph_clock;
        G.push_back(std::move(g));
        return;
    }
    it->last_use = ++ctx->graph_clock;
    if (!it->exec) {
        if (!ctx->capture_stream) KGF_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        KGF_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        hipStream_t saved = ctx->stream;
        ctx->stream = ctx->capture_stream;
        hipGraph_t graph = nullptr;
        try {
            sil_step_w(ctx, model, sec, psi, ncol, ld, o, w);
        } catch (...) {
            ctx->stream = saved;
            (void)hipStreamEndCapture(ctx->capture_stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        ctx->stream = saved;
        KGF_HIP(hipStreamEndCapture(ctx->capture_stream, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        KGF_HIP(e);
        it->exec = exec;
    }
    KGF_HIP(hipGraphLaunch(it->exec, ctx->stream));
}

void sil_propagate(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                   int nsteps, const SilOpts& o, double* err, double* drift) {
    TraceRange range_("kgf SIL steps");
    for (double* p : {err, drift})
        if (p && nsteps > 0) {
            hipLaunchKernelGGL(k_fill_zero, dim3((ncol + 255) / 256), dim3(256), 0, ctx->stream, p, ncol);
            check_launch("k_fill_zero");
        }
    for (int step = 0; step < nsteps; ++step) {
        KGF_REQUIRE(ncol <= 65535, KGF_EUNSUPPORTED, "SIL: at most 65535 columns per batch");
        hv_prepare(ctx, model, sec, ncol);
        sil_reserve(ctx, sec, ncol, o.m, o.reorth);
        SilWork w = sil_work_ws(ctx, sec, ncol, o);
        w.err = err;
        w.drift = drift;
        if (err)
            w.errc = static_cast<double2*>(
                workspace(ctx, "sil_errc", sizeof(double2) * (size_t)ncol * kErrNodes * o.m));
        if (ctx->use_graphs && !ctx->prof_on && !err && !drift)
            sil_step_graph(ctx, model, sec, psi, ncol, ld, o, w);
        else
            sil_step_w(ctx, model, sec, psi, ncol, ld, o, w);
    }
}

// Bytes of the single buffer a batched SIL step of ncol columns needs.
size_t sil_scratch_bytes(kgf_ctx* ctx, const kgf_sector* sec, int ncol, int m, int reorth) {
    return sil_layout(ctx, sec, ncol, m, reorth).total;
}

// SIL steps with every device buffer carved from `scratch` (at least
// sil_scratch_bytes); no allocation.  The hopping tables of the model for the
// sector's particle numbers must already exist.
double* sil_propagate_in(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                         int nsteps, const SilOpts& o, void* scratch, bool want_err) {
    const SilLayout l = sil_layout(ctx, sec, ncol, o.m, o.reorth);
    char* base = static_cast<char*>(scratch);
    SilWork w;
    w.X = reinterpret_cast<double2*>(base + l.x);
    w.scal = reinterpret_cast<double*>(base + l.scal);
    w.part = reinterpret_cast<double*>(base + l.part);
    w.part_big = o.reorth > 0 ? reinterpret_cast<double*>(base + l.part_big) : nullptr;
    w.hvec = o.reorth > 0 ? reinterpret_cast<double2*>(base + l.hvec) : nullptr;
    w.err = want_err ? reinterpret_cast<double*>(base + l.err) : nullptr;
    w.errc = want_err ? reinterpret_cast<double2*>(base + l.errc) : nullptr;
    w.drift = nullptr;
    if (w.err) {
        hipLaunchKernelGGL(k_fill_zero, dim3((ncol + 255) / 256), dim3(256), 0, ctx->stream, w.err, ncol);
        check_launch("k_fill_zero");
    }
    for (int step = 0; step < nsteps; ++step) sil_step_w(ctx, model, sec, psi, ncol, ld, o, w);
    return w.err;
}

// ---------------------------------------------------------------------------
// grouped launches: the columns of several instance groups (sectors of
// different size, a Hamiltonian per column) in every launch of a SIL step.
// Column c (blockIdx.y) reads its slots, dimension and partial area from
// cols[c]; per column the element-to-thread mapping, block count and
// reduction order are those of the single-group kernels above.
// ---------------------------------------------------------------------------
// column and block-within-column of a flattened streaming launch
__device__ __forceinline__ bool stream_block(const GroupRange* r, int ng, int64_t nblocks, int* c, int* bx) {
    const int64_t b = flat_block();
    if (b >= nblocks) return false;
    const int g = group_of_block(r, ng, b);
    const int64_t lb = b - r[g].blk0;
    *c = r[g].col0 + (int)(lb / r[g].nb);
    *bx = (int)(lb % r[g].nb);
    return true;
}

__global__ __launch_bounds__(kThreads) void k_norm2_groups(const GroupCol* __restrict__ cols,
                                                           const GroupRange* __restrict__ rg, int ng, int64_t nblocks) {
    __shared__ double sh[kThreads / 64];
    int c, bx;
    if (!stream_block(rg, ng, nblocks, &c, &bx)) return;
    const GroupCol C = cols[c];
    const double2* x = C.s0;
    double acc = 0.0;
    for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < C.D; i += (int64_t)C.nb * blockDim.x) {
        double2 z = x[i];
        acc = fma(z.x, z.x, acc);
        acc = fma(z.y, z.y, acc);
    }
    double v = block_sum(acc, sh);
    if (threadIdx.x == 0) C.part[bx] = v;
}

__global__ __launch_bounds__(kThreads) void k_update_groups(const GroupCol* __restrict__ cols,
                                                            const GroupRange* __restrict__ rg, int ng,
                                                            int64_t nblocks, int k, const double* __restrict__ scal) {
    __shared__ double sh[kThreads / 64];
    int c, bx;
    if (!stream_block(rg, ng, nblocks, &c, &bx)) return;
    const GroupCol C = cols[c];
    const double* sc = scal + (int64_t)c * kScalStride;
    const double f = sc[kOffA + k] * sc[kOffS + k];
    const double2* x = C.at(k);
    double2* y = C.at(k + 1);
    double acc = 0.0;
    for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < C.D; i += (int64_t)C.nb * blockDim.x) {
        double2 z = ld_once(x + i), w = y[i];
        w.x = fma(-f, z.x, w.x);
        w.y = fma(-f, z.y, w.y);
        y[i] = w;
        acc = fma(w.x, w.x, acc);
        acc = fma(w.y, w.y, acc);
    }
    double v = block_sum(acc, sh);
    if (threadIdx.x == 0) C.part[bx] = v;
}

__global__ __launch_bounds__(kThreads) void k_combine_groups(const GroupCol* __restrict__ cols,
                                                             const GroupRange* __restrict__ rg, int ng,
                                                             int64_t nblocks, int n, const double* __restrict__ scal) {
    extern __shared__ double2 cf[];
    int c, bx;
    if (!stream_block(rg, ng, nblocks, &c, &bx)) return;
    const GroupCol C = cols[c];
    const double2* coef = reinterpret_cast<const double2*>(scal + (int64_t)c * kScalStride + kOffCoef);
    for (int j = threadIdx.x; j < n; j += blockDim.x) cf[j] = coef[j];
    __syncthreads();
    double2* o = C.s0;
    for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < C.D; i += (int64_t)C.nb * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; ++j) {
            const double2 z = ld_once(C.at(j) + i);
            const double2 h = cf[j];
            re = fma(h.x, z.x, fma(-h.y, z.y, re));
            im = fma(h.x, z.y, fma(h.y, z.x, im));
        }
        o[i] = make_double2(re, im);
    }
}

// workspace sizes of a grouped SIL step: Krylov slots, partials
static void group_sizes(const std::vector<GroupSpec>& groups, int m, size_t* xbytes, size_t* pbytes, int* ncol) {
    *xbytes = *pbytes = 0;
    *ncol = 0;
    for (const GroupSpec& g : groups) {
        const int64_t D = g.sec->dim();
        *ncol += g.ncol;
        *xbytes += sizeof(double2) * (size_t)m * g.ncol * D;
        *pbytes += sizeof(double) * (size_t)g.ncol * std::max<int64_t>(red_blocks(D), g.sec->d_up);
    }
}

void sil_groups_reserve(kgf_ctx* ctx, const std::vector<GroupSpec>& groups, int m) {
    size_t xbytes, pbytes;
    int ncol;
    group_sizes(groups, m, &xbytes, &pbytes, &ncol);
    auto& xs = ctx->ws["sg_X"];
    if (!xs || xs->bytes < xbytes) {
        if (xs) {
            sync(ctx);
            xs.reset();
        }
        ensure_device_fits(xbytes, "grouped SIL Krylov basis");
        workspace(ctx, "sg_X", xbytes);
    }
    workspace(ctx, "sg_part", pbytes);
    workspace(ctx, "sg_scal", sizeof(double) * kScalStride * (size_t)std::max(ncol, 1));
}

void sil_step_groups(kgf_ctx* ctx, const std::vector<GroupSpec>& groups, const std::vector<double2*>& psi,
                     const std::vector<int64_t>& ld, const SilOpts& o) {
    KGF_REQUIRE(o.reorth == 0, KGF_EUNSUPPORTED, "grouped SIL step: no reorthogonalisation");
    const int m = o.m;
    int ncol = 0;
    for (const GroupSpec& g : groups) {
        KGF_REQUIRE(g.col0 == ncol, KGF_EINVAL, "grouped SIL step: groups must take consecutive columns");
        ncol += g.ncol;
    }
    if (ncol == 0) return;
    KGF_REQUIRE(ncol <= 65535, KGF_EUNSUPPORTED, "grouped SIL step: at most 65535 columns");
    size_t xbytes, pbytes;
    group_sizes(groups, m, &xbytes, &pbytes, &ncol);
    sil_groups_reserve(ctx, groups, m);   // a no-op when the caller reserved the largest step beforehand
    char* X = static_cast<char*>(workspace(ctx, "sg_X", xbytes));
    double* part = static_cast<double*>(workspace(ctx, "sg_part", pbytes));
    double* scal = static_cast<double*>(workspace(ctx, "sg_scal", sizeof(double) * kScalStride * (size_t)ncol));
    std::vector<GroupCol> cols((size_t)ncol);
    size_t xo = 0, po = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const GroupSpec& g = groups[gi];
        const int64_t D = g.sec->dim();
        double2* Xg = reinterpret_cast<double2*>(X + xo);
        for (int lc = 0; lc < g.ncol; ++lc) {
            GroupCol& C = cols[(size_t)g.col0 + lc];
            C.s0 = psi[gi] + (int64_t)lc * ld[gi];
            C.X1 = Xg + (int64_t)lc * D;
            C.x_slot = (int64_t)g.ncol * D;
            C.D = D;
            C.part = part + po;
            C.group = (int)gi;
            C.nb = red_blocks(D);
            C.nrow = (int)g.sec->d_up;
            po += (size_t)std::max<int64_t>(C.nb, g.sec->d_up);
        }
        xo += sizeof(double2) * (size_t)m * g.ncol * D;
    }
    // block ranges of the flattened streaming launches (nb blocks per column)
    std::vector<GroupRange> ranges;
    int64_t nstream = 0;
    for (const GroupSpec& g : groups) {
        if (g.ncol == 0) continue;
        GroupRange r;
        r.blk0 = nstream;
        r.nb = red_blocks(g.sec->dim());
        r.col0 = g.col0;
        nstream += (int64_t)r.nb * g.ncol;
        ranges.push_back(r);
    }
    const int ng = (int)ranges.size();
    // upload the column and range tables when they changed (a sweep keeps them for many steps)
    const size_t cb = sizeof(GroupCol) * cols.size(), rb = sizeof(GroupRange) * ranges.size();
    std::vector<unsigned char> hb(cb + rb);
    std::memcpy(hb.data(), cols.data(), cb);
    std::memcpy(hb.data() + cb, ranges.data(), rb);
    if (!ctx->ws.count("sg_cols") || ctx->gcol_table != hb) {
        upload_table(ctx, "sg_cols", hb.data(), hb.size());
        ctx->gcol_table = std::move(hb);
    }
    const GroupCol* dcols = static_cast<const GroupCol*>(ctx->ws["sg_cols"]->p);
    const GroupRange* drng = reinterpret_cast<const GroupRange*>(static_cast<char*>(ctx->ws["sg_cols"]->p) + cb);
    static_assert(sizeof(GroupCol) % alignof(GroupRange) == 0, "range table alignment");
    double vec = 0.0;
    for (const GroupSpec& g : groups) vec += 16.0 * (double)g.sec->dim() * g.ncol;
    {
        Prof pr(ctx, "norm", vec);
        hipLaunchKernelGGL(k_norm2_groups, flat_grid(nstream), dim3(kThreads), 0, ctx->stream, dcols, drng, ng, nstream);
        check_launch("k_norm2_groups");
    }
    auto fin = [&](int mode, int k, int rows, double tol) {
        Prof pr(ctx, "fin");
        hipLaunchKernelGGL(k_fin_groups, dim3(ncol), dim3(kThreads), 0, ctx->stream, mode, k, dcols, rows, scal, tol);
        check_launch("k_fin_groups");
    };
    fin(FIN_INIT, 0, 0, 0.0);
    for (int k = 0; k < m; ++k) {
        hv_lanczos_groups(ctx, groups, dcols, ncol, k, scal, kScalStride);
        fin(FIN_A, k, 1, 0.0);
        if (k == m - 1) break;
        {
            Prof pr(ctx, "lanczos_update", 3.0 * vec);
            hipLaunchKernelGGL(k_update_groups, flat_grid(nstream), dim3(kThreads), 0, ctx->stream, dcols, drng, ng,
                               nstream, k, scal);
            check_launch("k_update_groups");
        }
        fin(FIN_B, k, 0, o.breakdown_tol);
    }
    double2* coef = reinterpret_cast<double2*>(scal + kOffCoef);
    for (int r0 = 0; r0 < ncol; r0 += kMaxReq) {
        CoefReq q;
        q.n = std::min(kMaxReq, ncol - r0);
        for (int r = 0; r < q.n; ++r) {
            q.col[r] = r0 + r;
            q.t[r] = o.dt;
            q.dir[r] = o.direction;
        }
        launch_coefs(ctx, scal, m, q, o.shift, coef + (int64_t)r0 * (kScalStride / 2), kScalStride / 2);
    }
    Prof pr(ctx, "combine", (m + 1) * vec);
    hipLaunchKernelGGL(k_combine_groups, flat_grid(nstream), dim3(kThreads), sizeof(double2) * m, ctx->stream, dcols,
                       drng, ng, nstream, m, scal);
    check_launch("k_combine_groups");
}

// Uniqueness of a ground state: a second recursion from a SplitMix64 start
// vector (entry i: output i of the generator seeded with `seed`, mapped to
// [-1, 1)), and |<psi0|psi_b>|^2 of the two normalised Ritz vectors.
__global__ void k_splitmix_fill(double2* __restrict__ v, int64_t D, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * 0x1.0p-53;
        v[i] = make_double2(2.0 * u - 1.0, 0.0);
    }
}

void fill_splitmix(kgf_ctx* ctx, double2* v, int64_t n, uint64_t seed) {
    const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_splitmix_fill, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), 0, ctx->stream,
                       v, n, seed);
    check_launch("k_splitmix_fill");
}

// Sweep block width by measurement (KGF_OPT_HV_TUNE): one batched SIL step
// on scratch columns at each candidate width up to max_cols (the widest that
// fits, then 32, 16, 8, 4), timed with HIP events after a warm-up step.  The
// widest candidate within 5% of the best column-steps per second is kept for
// the sector shape and Krylov options: a narrower block means more chunks,
// each starting with a growth phase of narrow blocks, which one step does not
// see.  Column results do not depend on the width.
int tuned_sweep_width(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int max_cols, const SilOpts& o) {
    const std::array<int, 4> key = {sec->L, sec->n_up * 64 + sec->n_dn, o.m, o.reorth};
    auto it = ctx->sweep_tuned.find(key);
    if (it != ctx->sweep_tuned.end()) return std::min(it->second, max_cols);
    const int64_t D = sec->dim();
    std::vector<int> cand;
    for (int c : {max_cols, 32, 16, 8, 4})
        if (c >= 1 && c <= max_cols && std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    if (cand.size() <= 1 || D == 0) {
        ctx->sweep_tuned[key] = max_cols;
        return max_cols;
    }
    ensure_device_fits(sizeof(double2) * (size_t)max_cols * D, "sweep width tuning columns");
    double2* X = static_cast<double2*>(workspace(ctx, "tune_cols", sizeof(double2) * (size_t)max_cols * D));
    fill_splitmix(ctx, X, (int64_t)max_cols * D, 0x5eedULL);
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    hipEvent_t e0, e1;
    KGF_HIP(hipEventCreate(&e0));
    KGF_HIP(hipEventCreate(&e1));
    std::vector<double> rate(cand.size());
    double best_rate = 0.0;
    for (size_t i = 0; i < cand.size(); ++i) {
        const int c = cand[i];
        sil_propagate(ctx, model, sec, X, c, D, 1, o);   // warm-up (tables, workspaces, graph bookkeeping)
        KGF_HIP(hipEventRecord(e0, ctx->stream));
        sil_propagate(ctx, model, sec, X, c, D, 1, o);
        KGF_HIP(hipEventRecord(e1, ctx->stream));
        KGF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        KGF_HIP(hipEventElapsedTime(&ms, e0, e1));
        rate[i] = c / std::max(1e-6, (double)ms);
        best_rate = std::max(best_rate, rate[i]);
    }
    int best = cand.back();
    for (size_t i = 0; i < cand.size(); ++i)   // candidates run from the widest down
        if (rate[i] >= 0.95 * best_rate) {
            best = cand[i];
            break;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof_on = prof;
    release_ws(ctx, "tune_cols");
    ctx->sweep_tuned[key] = best;
    return best;
}

double gs_fidelity2(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0,
                    const kgf_gs_opts* o) {
    const int64_t D = sec->dim();
    double2* v = static_cast<double2*>(workspace(ctx, "gs_chk_v", sizeof(double2) * (size_t)D));
    const int64_t blocks = std::min<int64_t>((D + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_splitmix_fill, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), 0,
                       ctx->stream, v, D, o->unique_seed);
    check_launch("k_splitmix_fill");
    ground_state(ctx, model, sec, v, v, o->tol, o->max_iter, o->check_every, o->reorth);   // psi_b over its start
    double2* dd = static_cast<double2*>(workspace(ctx, "gs_chk_dot", sizeof(double2)));
    block_dots(ctx, psi0, D, 1, v, D, 1, D, dd);
    double2 h;
    KGF_HIP(hipMemcpyAsync(&h, dd, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    ctx->ws.erase("gs_chk_v");
    ctx->ws.erase("gs_V");
    return h.x * h.x + h.y * h.y;
}

void require_unique_ground_state(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0,
                                 const kgf_gs_opts* o, const char* who) {
    if (!o || !o->unique_check) return;
    const double f2 = gs_fidelity2(ctx, model, sec, psi0, o);
    const double tol = o->unique_tol > 0.0 ? o->unique_tol : 1e-10;
    if (!(f2 >= 1.0 - tol))
        fail(KGF_EDEGENERATE, std::string(who) + ": the ground state of H_ini is not unique (two Lanczos starts give "
                                                 "|<0_a|0_b>|^2 = " + std::to_string(f2) + ")");
}


// ---------------------------------------------------------------------------
// ground state
// ---------------------------------------------------------------------------
// One Lanczos run of at most max_iter steps from v0; the Ritz vector of the
// lowest Ritz value goes to psi0 (normalised).  psi0 may alias v0.
static GsResult gs_cycle(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* v0,
                         double2* psi0, double tol, int max_iter, int check_every, int reorth) {
    const int64_t D = sec->dim();
    hv_prepare(ctx, model, sec);
    const int nmax = max_iter + 1;
    const size_t vbytes = sizeof(double2) * (size_t)nmax * D;
    auto& xs = ctx->ws["gs_V"];
    if (!xs || xs->bytes < vbytes) ensure_device_fits(vbytes - (xs ? xs->bytes : 0), "ground-state Lanczos basis");
    double2* V = static_cast<double2*>(workspace(ctx, "gs_V", vbytes));
    double* a = static_cast<double*>(workspace(ctx, "gs_a", sizeof(double) * (nmax + 1)));
    double* b = static_cast<double*>(workspace(ctx, "gs_b", sizeof(double) * (nmax + 1)));
    double* s = static_cast<double*>(workspace(ctx, "gs_s", sizeof(double) * (nmax + 1)));
    double* y = static_cast<double*>(workspace(ctx, "gs_y", sizeof(double) * (nmax + 1)));
    double* scratch = static_cast<double*>(workspace(ctx, "gs_scratch", sizeof(double) * 6 * (nmax + 1)));
    double* res = static_cast<double*>(workspace(ctx, "gs_res", sizeof(double) * 8));
    double2* coef = static_cast<double2*>(workspace(ctx, "gs_coef", sizeof(double2) * (nmax + 1)));
    const int NB = red_blocks(D);
    const int HB = hv_lanczos_blocks(ctx, sec);
    double* part = static_cast<double*>(workspace(ctx, "gs_part", sizeof(double) * (NB > HB ? NB : HB)));
    double* part_big = static_cast<double*>(workspace(ctx, "gs_partbig", sizeof(double) * (size_t)NB * 2 * (nmax + 1)));
    double2* hvec = static_cast<double2*>(workspace(ctx, "gs_hvec", sizeof(double2) * (nmax + 1)));
    double* host = static_cast<double*>(host_scratch(ctx, sizeof(double) * 8));
    Slots sl{V, 0, V + D, D, 0};

    KGF_HIP(hipMemcpyAsync(V, v0, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
    {
        Prof pr(ctx, "norm");
        hipLaunchKernelGGL(k_norm2, dim3(NB, 1), dim3(kThreads), 0, ctx->stream, V, D, D, part);
        check_launch("k_norm2");
    }
    hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_INIT, 0, part, NB, a, b, s);
    check_launch("k_gs_fin");

    GsResult out{0.0, 0, false, INFINITY};
    int n = 0;
    for (int k = 0; k < max_iter; ++k) {
        LanczosHvArgs ha;
        ha.x = sl.at(k, 0);
        ha.x_col = 0;
        ha.xp = k > 0 ? sl.at(k - 1, 0) : nullptr;
        ha.xp_col = 0;
        ha.y = sl.at(k + 1, 0);
        ha.y_col = 0;
        ha.s_k = s + k;
        ha.b_k = b + k;
        ha.s_km1 = s + (k > 0 ? k - 1 : 0);
        ha.stride = 0;
        ha.part = part;
        hv_lanczos(ctx, model, sec, 1, ha);
        hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_A, k, part, HB, a, b, s);
        check_launch("k_gs_fin");
        {
            Prof pr(ctx, "lanczos_update");
            hipLaunchKernelGGL(k_update, dim3(NB, 1), dim3(kThreads), 0, ctx->stream, sl, k, a + k, s + k, 0,
                               D, part);
            check_launch("k_update");
        }
        if (reorth > 0)
            reorthogonalise(ctx, sl, k + 1, k + 1, 1, D, reorth, nullptr, s, part, part_big, hvec);
        hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_B, k, part, NB, a, b, s);
        check_launch("k_gs_fin");
        n = k + 1;
        if ((k + 1) % check_every == 0 || k == max_iter - 1) {
            {
                Prof pr(ctx, "gs_eig");
                hipLaunchKernelGGL(k_gs_eig, dim3(1), dim3(64), 0, ctx->stream, a, b, n, scratch, y, res);
                check_launch("k_gs_eig");
            }
            KGF_HIP(hipMemcpyAsync(host, res, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            out.E0 = host[0];
            out.residual = host[1];
            out.iters = (int)host[2];
            if (ctx->progress) ctx->progress(ctx->progress_user, "ground_state", k + 1, max_iter);
            if (host[3] != 0.0 || host[1] <= tol * fmax(1.0, fabs(host[0]))) {
                out.converged = true;
                break;
            }
        }
    }
    // Ritz vector psi0 = sum_j y_j s_j x_j, then normalise
    const int ne = out.iters > 0 ? out.iters : n;
    hipLaunchKernelGGL(k_gs_coef, dim3(1), dim3(kThreads), 0, ctx->stream, y, s, ne, coef);
    check_launch("k_gs_coef");
    {
        Prof pr(ctx, "combine");
        hipLaunchKernelGGL(k_combine, dim3(NB, 1), dim3(kThreads), sizeof(double2) * ne, ctx->stream, sl, ne,
                           coef, (int64_t)0, psi0, (int64_t)0, D);
        check_launch("k_combine");
    }
    hipLaunchKernelGGL(k_norm2, dim3(NB, 1), dim3(kThreads), 0, ctx->stream, psi0, D, D, part);
    check_launch("k_norm2");
    hipLaunchKernelGGL(k_inv_sqrt, dim3(1), dim3(kThreads), 0, ctx->stream, part, NB, res + 4);
    check_launch("k_inv_sqrt");
    hipLaunchKernelGGL(k_scale, dim3(NB), dim3(kThreads), 0, ctx->stream, psi0, D, res + 4);
    check_launch("k_scale");
    sync(ctx);
    return out;
}

// The tridiagonal Lanczos matrix of n steps from i0 (Eqs. (recursion),
// (tmatrix)): a[0..n), b[1..n) on the host (b[k] couples steps k-1 and k),
// norm2 = <i0|i0>.  The basis is kept for the reorthogonalisation (passes
// 0..2).  Returns the number of steps taken: fewer than n when the Krylov
// space is exhausted (b = 0), after which the matrix is exact.
int lanczos_tridiag(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* i0, int n, int reorth,
                    double* a_host, double* b_host, double* norm2_host) {
    const int64_t D = sec->dim();
    hv_prepare(ctx, model, sec);
    const size_t vbytes = sizeof(double2) * (size_t)(n + 1) * D;
    ensure_device_fits(vbytes, "Lanczos basis");
    double2* V = static_cast<double2*>(workspace(ctx, "lt_V", vbytes));
    double* a = static_cast<double*>(workspace(ctx, "lt_a", sizeof(double) * (n + 2)));
    double* b = static_cast<double*>(workspace(ctx, "lt_b", sizeof(double) * (n + 2)));
    double* s = static_cast<double*>(workspace(ctx, "lt_s", sizeof(double) * (n + 2)));
    const int NB = red_blocks(D);
    const int HB = hv_lanczos_blocks(ctx, sec);
    double* part = static_cast<double*>(workspace(ctx, "lt_part", sizeof(double) * (NB > HB ? NB : HB)));
    double* part_big = static_cast<double*>(workspace(ctx, "lt_partbig", sizeof(double) * (size_t)NB * 2 * (n + 2)));
    double2* hvec = static_cast<double2*>(workspace(ctx, "lt_hvec", sizeof(double2) * (n + 2)));
    Slots sl{V, 0, V + D, D, 0};
    KGF_HIP(hipMemcpyAsync(V, i0, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_norm2, dim3(NB, 1), dim3(kThreads), 0, ctx->stream, V, D, D, part);
    check_launch("k_norm2");
    double2* n2dev = static_cast<double2*>(workspace(ctx, "lt_n2", sizeof(double2)));
    hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_INIT, 0, part, NB, a, b, s);
    check_launch("k_gs_fin");
    block_dots(ctx, V, D, 1, V, D, 1, D, n2dev);
    for (int k = 0; k < n; ++k) {
        LanczosHvArgs ha;
        ha.x = sl.at(k, 0);
        ha.x_col = 0;
        ha.xp = k > 0 ? sl.at(k - 1, 0) : nullptr;
        ha.xp_col = 0;
        ha.y = sl.at(k + 1, 0);
        ha.y_col = 0;
        ha.s_k = s + k;
        ha.b_k = b + k;
        ha.s_km1 = s + (k > 0 ? k - 1 : 0);
        ha.stride = 0;
        ha.part = part;
        hv_lanczos(ctx, model, sec, 1, ha);
        hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_A, k, part, HB, a, b, s);
        check_launch("k_gs_fin");
        if (k == n - 1) break;
        hipLaunchKernelGGL(k_update, dim3(NB, 1), dim3(kThreads), 0, ctx->stream, sl, k, a + k, s + k, 0, D, part);
        check_launch("k_update");
        if (reorth > 0) reorthogonalise(ctx, sl, k + 1, k + 1, 1, D, reorth, nullptr, s, part, part_big, hvec);
        hipLaunchKernelGGL(k_gs_fin, dim3(1), dim3(kThreads), 0, ctx->stream, (int)FIN_B, k, part, NB, a, b, s);
        check_launch("k_gs_fin");
    }
    std::vector<double> ha(n + 2), hb(n + 2), hs(n + 2);
    double2 n2;
    KGF_HIP(hipMemcpyAsync(ha.data(), a, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, ctx->stream));
    KGF_HIP(hipMemcpyAsync(hb.data(), b, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, ctx->stream));
    KGF_HIP(hipMemcpyAsync(hs.data(), s, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, ctx->stream));
    KGF_HIP(hipMemcpyAsync(&n2, n2dev, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    int taken = 0;
    while (taken < n && hs[taken] != 0.0) ++taken;   // s_k = 0 once the space is exhausted
    for (int k = 0; k < n; ++k) {
        a_host[k] = k < taken ? ha[k] : 0.0;
        b_host[k] = (k >= 1 && k < taken) ? hb[k] : 0.0;
    }
    *norm2_host = n2.x;
    for (const char* nm : {"lt_V", "lt_partbig"}) ctx->ws.erase(nm);
    return taken;
}

// Ground state of H in the sector.  When the Lanczos basis of max_iter + 1
// vectors does not fit in device memory (large sectors), the recursion is
// restarted from the current Ritz vector every `cap` vectors (explicit
// restart); the iteration count and the stopping rule are unchanged.
GsResult ground_state(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* v0,
                      double2* psi0, double tol, int max_iter, int check_every, int reorth) {
    TraceRange range_("kgf ground state");
    const int64_t D = sec->dim();
    const size_t vbytes = sizeof(double2) * (size_t)D;
    size_t free_b = 0, total_b = 0;
    KGF_HIP(hipMemGetInfo(&free_b, &total_b));
    auto it = ctx->ws.find("gs_V");
    const size_t have = it != ctx->ws.end() && it->second ? it->second->bytes : 0;
    const size_t budget = have + (size_t)(0.7 * (double)free_b);
    int64_t cap = (int64_t)(budget / std::max<size_t>(vbytes, 1));
    if (ctx->gs_max_basis > 0) cap = std::min<int64_t>(cap, ctx->gs_max_basis);
    if (cap >= max_iter + 1) return gs_cycle(ctx, model, sec, v0, psi0, tol, max_iter, check_every, reorth);
    KGF_REQUIRE(cap >= 8, KGF_ENOMEM, "ground state: fewer than 8 Lanczos vectors fit in device memory");
    const int len = (int)std::min<int64_t>(cap - 1, 4096);
    GsResult out{0.0, 0, false, INFINITY};
    const double2* start = v0;
    int done = 0;
    while (done < max_iter) {
        const int k = std::min(len, max_iter - done);
        GsResult r = gs_cycle(ctx, model, sec, start, psi0, tol, k, std::min(check_every, k), reorth);
        done += r.iters > 0 ? r.iters : k;
        out.E0 = r.E0;
        out.residual = r.residual;
        out.iters = done;
        if (r.converged) {
            out.converged = true;
            break;
        }
        start = psi0;
    }
    return out;
}

// ---------------------------------------------------------------------------
// block dots
// ---------------------------------------------------------------------------
void block_dots(kgf_ctx* ctx, const double2* Lv, int64_t l_col, int nl, const double2* Rv, int64_t r_col,
                int nr, int64_t D, double2* out, int64_t out_ld) {
    if (nl == 0 || nr == 0) return;
    if (out_ld <= 0) out_ld = nr;
    const int NB = red_blocks(D) < 256 ? red_blocks(D) : 256;
    double* part = static_cast<double*>(workspace(ctx, "dots_part", sizeof(double) * (size_t)NB * nl * nr * 2));
    const int nchunk = (nl + kDotChunk - 1) / kDotChunk;
    KGF_REQUIRE(nr <= 65535 && nchunk <= 65535 && (int64_t)nl * nr <= 0x7fffffff, KGF_EUNSUPPORTED,
                "dots: too many vectors");
    {
        Prof pr(ctx, "dots");
        hipLaunchKernelGGL(k_dots, dim3(NB, nr, nchunk), dim3(kThreads), 0, ctx->stream, Lv, l_col, nl, Rv,
                           r_col, (const double2* const*)nullptr, D, part);
        check_launch("k_dots");
    }
    hipLaunchKernelGGL(k_dots_fin, dim3(nl * nr), dim3(kThreads), 0, ctx->stream, part, NB, nr, out_ld, out);
    check_launch("k_dots_fin");
}

}  // namespace kgf
