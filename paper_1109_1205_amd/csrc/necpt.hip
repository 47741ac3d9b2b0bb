// Nonequilibrium cluster-perturbation theory (Sec. 5, Eq. (cpteq)) on the
// Keldysh contour.  The CPT equation G = (G'^-1 - V)^-1 for a cluster whose
// site b is linked by the hopping V to site 1 of an uncorrelated bath reduces,
// on the cluster, to G = G^c + G^c * Sigma * G with the embedding function
// Sigma(z, z') = V^2 G^b_11(z, z') acting on site b only (the bath block is
// eliminated exactly, also after discretisation).  Row b is solved first,
//     (1 - G^c_bb K) X_j = G^c_bj,   K(p, q) = w_p Sigma(z_p, z_q) w_q,
// then G_ij = G^c_ij + G^c_ib K X_j.
// Contour: the mesh t_k = k dt, k < nt, forward (points p = k) then backward
// (p = 2nt-1-k); a contour function takes G^> where z is later than z', G^<
// where earlier; the contour integral is the trapezoid rule on each branch
// (weights +dt forward, -dt backward, halved at the ends of each branch) with
// the integrand's jumps at nodes.  On the equal-point diagonal an interior
// node takes the mean (G^> + G^<)/2; a branch end takes the limit from inside
// its branch, which depends on where the matrix enters: as the kernel
// G(z, z'') ("row": G^< at a branch start, G^> at a branch end) or as the
// right-hand side, whose diagonal becomes the unknown's and is later used
// as G(z'', z') ("rhs": the other way round).  This makes the scheme second
// order in dt (first order with the mean at the ends as well).  Dense complex
// FP64 algebra: an LDS-tiled GEMM and a right-looking LU with partial pivoting.
//
// With an imaginary branch (Sec. 5: the initial state of the connected
// system is treated by CPT too, through a Matsubara branch of length beta)
// the contour gets ntau more points z = -i tau_j, tau_j = j dtau, later than
// both real branches, with the weight -i dtau (halved at its ends) and the
// same equal-point rules; a contour function then also takes its mixed
// components G^<(t, -i tau) (real point earlier), G^>(-i tau, t) and its
// imaginary-branch functions of tau - tau'.
#include <cmath>
#include <vector>

#include "kgf_internal.h"

namespace kgf {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// contour point p: branch 0 forward (t_p), 1 backward (t_{2nt-1-p}), 2 imaginary (tau_{p-2nt})
__device__ __forceinline__ int cbranch(int p, int nt) { return p < nt ? 0 : (p < 2 * nt ? 1 : 2); }
__device__ __forceinline__ int cindex(int p, int nt) { return p < nt ? p : (p < 2 * nt ? 2 * nt - 1 - p : p - 2 * nt); }

// quadrature weight: +-dt on the real branches, -i dtau on the imaginary one,
// halved at the ends of each branch
__device__ __forceinline__ double2 cweight(int p, int nt, int ntau, double dt, double dtau) {
    const int b = cbranch(p, nt), k = cindex(p, nt);
    if (b < 2) {
        const double w = (nt > 1) ? ((k == 0 || k == nt - 1) ? 0.5 * dt : dt) : 0.0;
        return make_double2(b == 0 ? w : -w, 0.0);
    }
    const double w = (ntau > 1) ? ((k == 0 || k == ntau - 1) ? 0.5 * dtau : dtau) : 0.0;
    return make_double2(0.0, -w);
}

// One orbital pair of a contour function: element pointers and mesh strides
// (lesser / greater [a][b], mixed [a][j] = G^<(t_a, -i tau_j), mixed_left
// [j][b] = G^>(-i tau_j, t_b), vertical [d]: G^>(-i tau_{j+d}, -i tau_j) and
// G^<(-i tau_j, -i tau_{j+d})).  The imaginary parts are null without a
// Matsubara branch.
struct CFn {
    const double2 *l, *g, *mx, *mxl, *vg, *vl;
    int64_t la, lb, ma, mj, xj, xb, vd;
};

// out[p * ldo + q] = s * (weights ? w_p w_q : 1) * G(z_p, z_q); rhs = 0: row
// values at the branch ends, 1: right-hand-side values
__global__ void k_to_contour(CFn f, int nt, int ntau, double s, int weights, int rhs, double dt, double dtau,
                             double2* __restrict__ out, int64_t ldo) {
    const int n = 2 * nt + ntau;
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / n), q = (int)(e % n);
        const int bp = cbranch(p, nt), bq = cbranch(q, nt);
        const int a = cindex(p, nt), b = cindex(q, nt);
        double2 v;
        if (bp == 2 && bq < 2) {
            v = f.mxl[a * f.xj + b * f.xb];
        } else if (bp < 2 && bq == 2) {
            v = f.mx[a * f.ma + b * f.mj];
        } else {
            double2 gg, gl;   // the two orderings at (p, q); only the valid one is read
            if (bp < 2) {
                const int64_t off = a * f.la + b * f.lb;
                if (p >= q) gg = f.g[off];
                if (p <= q) gl = f.l[off];
            } else {
                if (a >= b) gg = f.vg[(a - b) * f.vd];
                if (a <= b) gl = f.vl[(b - a) * f.vd];
            }
            const bool real_end = nt > 1 && (p == 0 || p == nt || p == nt - 1 || p == 2 * nt - 1);
            const bool tau_end = ntau > 1 && (p == 2 * nt || p == n - 1);
            if (p > q) {
                v = gg;
            } else if (p < q) {
                v = gl;
            } else if (real_end || tau_end) {
                const bool start = p == 0 || p == nt || p == 2 * nt;   // first point of its branch
                v = (start != (rhs != 0)) ? gl : gg;
            } else {
                v = make_double2(0.5 * (gg.x + gl.x), 0.5 * (gg.y + gl.y));
            }
        }
        double2 fct = make_double2(s, 0.0);
        if (weights) fct = cmul(fct, cmul(cweight(p, nt, ntau, dt, dtau), cweight(q, nt, ntau, dt, dtau)));
        out[p * ldo + q] = cmul(fct, v);
    }
}

__global__ void k_identity(double2* __restrict__ A, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        A[e] = make_double2((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
}

// C = alpha A B + beta C, row-major complex; 64x64 tile per 256-thread block,
// thread (ty, tx) owns rows ty + 16 r and columns tx + 16 c, r, c < 4.
constexpr int kGT = 64, kGK = 8;

__global__ void __launch_bounds__(256) k_zgemm(int M, int N, int K, double2 alpha, const double2* __restrict__ A,
                                               int64_t lda, const double2* __restrict__ B, int64_t ldb, double2 beta,
                                               double2* __restrict__ C, int64_t ldc) {
    __shared__ double2 As[kGK][kGT];
    __shared__ double2 Bs[kGK][kGT];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int row0 = blockIdx.y * kGT, col0 = blockIdx.x * kGT;
    double2 acc[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < K; k0 += kGK) {
        for (int e = tid; e < kGT * kGK; e += 256) {
            const int r = e / kGK, k = e % kGK;          // A tile: 64 rows x 8
            const int gr = row0 + r, gk = k0 + k;
            As[k][r] = (gr < M && gk < K) ? A[gr * lda + gk] : make_double2(0.0, 0.0);
            const int kb = e / kGT, cb = e % kGT;        // B tile: 8 rows x 64
            const int gkb = k0 + kb, gc = col0 + cb;
            Bs[kb][cb] = (gkb < K && gc < N) ? B[gkb * ldb + gc] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int k = 0; k < kGK; ++k) {
            double2 a[4], b[4];
            for (int r = 0; r < 4; ++r) a[r] = As[k][ty + 16 * r];
            for (int c = 0; c < 4; ++c) b[c] = Bs[k][tx + 16 * c];
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    acc[r][c].x = fma(a[r].x, b[c].x, fma(-a[r].y, b[c].y, acc[r][c].x));
                    acc[r][c].y = fma(a[r].x, b[c].y, fma(a[r].y, b[c].x, acc[r][c].y));
                }
        }
        __syncthreads();
    }
    const bool use_c = beta.x != 0.0 || beta.y != 0.0;
    for (int r = 0; r < 4; ++r) {
        const int gr = row0 + ty + 16 * r;
        if (gr >= M) continue;
        for (int c = 0; c < 4; ++c) {
            const int gc = col0 + tx + 16 * c;
            if (gc >= N) continue;
            double2 v = cmul(alpha, acc[r][c]);
            if (use_c) {
                const double2 o = cmul(beta, C[gr * ldc + gc]);
                v.x += o.x;
                v.y += o.y;
            }
            C[gr * ldc + gc] = v;
        }
    }
}

void zgemm(kgf_ctx* ctx, int M, int N, int K, double2 alpha, const double2* A, int64_t lda, const double2* B,
           int64_t ldb, double2 beta, double2* C, int64_t ldc) {
    if (M == 0 || N == 0) return;
    const dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
    Prof pr(ctx, "k_zgemm");
    hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, ctx->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    check_launch("k_zgemm");
}

// LU step k, part 1 (one block): pivot row = argmax_{i >= k} |A[i][k]|,
// swapped with row k in A (n columns) and B (m columns); |pivot| -> piv[k].
__global__ void __launch_bounds__(256) k_lu_pivot(double2* __restrict__ A, int n, double2* __restrict__ B, int m,
                                                  int k, double* __restrict__ piv) {
    __shared__ double sv[256];
    __shared__ int si[256];
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = A[(int64_t)i * n + k];
        const double v = a.x * a.x + a.y * a.y;
        if (v > best) {
            best = v;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = sv[threadIdx.x + s];
            const int oi = si[threadIdx.x + s];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = si[0];
    if (threadIdx.x == 0) piv[k] = sqrt(sv[0] > 0.0 ? sv[0] : 0.0);
    if (p != k) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double2 t = A[(int64_t)k * n + j];
            A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
            A[(int64_t)p * n + j] = t;
        }
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            const double2 t = B[(int64_t)k * m + j];
            B[(int64_t)k * m + j] = B[(int64_t)p * m + j];
            B[(int64_t)p * m + j] = t;
        }
    }
}

// LU step k, part 2: rows i > k of [A | B] minus (A[i][k] / A[k][k]) row k,
// columns > k of A and all of B (column k and row k are only read).
__global__ void k_lu_elim(double2* __restrict__ A, int n, double2* __restrict__ B, int m, int k) {
    const int w = (n - k - 1) + m;
    const int64_t total = (int64_t)(n - k - 1) * w;
    const double2 d = A[(int64_t)k * n + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 dinv = make_double2(d.x / dd, -d.y / dd);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = k + 1 + (int)(e / w);
        const int c = (int)(e % w);
        const double2 l = cmul(A[(int64_t)i * n + k], dinv);
        double2* dst;
        double2 src;
        if (c < n - k - 1) {
            const int j = k + 1 + c;
            dst = A + (int64_t)i * n + j;
            src = A[(int64_t)k * n + j];
        } else {
            const int j = c - (n - k - 1);
            dst = B + (int64_t)i * m + j;
            src = B[(int64_t)k * m + j];
        }
        const double2 t = cmul(l, src);
        *dst = make_double2(dst->x - t.x, dst->y - t.y);
    }
}

// back substitution step k: rows i < k of B minus A[i][k] x_k, x_k = B[k] / A[k][k]
__global__ void k_lu_back(const double2* __restrict__ A, int n, double2* __restrict__ B, int m, int k) {
    const int64_t total = (int64_t)k * m;
    const double2 d = A[(int64_t)k * n + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 dinv = make_double2(d.x / dd, -d.y / dd);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / m), j = (int)(e % m);
        const double2 x = cmul(B[(int64_t)k * m + j], dinv);
        const double2 t = cmul(A[(int64_t)i * n + k], x);
        B[(int64_t)i * m + j] = make_double2(B[(int64_t)i * m + j].x - t.x, B[(int64_t)i * m + j].y - t.y);
    }
}

__global__ void k_lu_scale(const double2* __restrict__ A, int n, double2* __restrict__ B, int m) {
    const int64_t total = (int64_t)n * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / m);
        const double2 d = A[(int64_t)i * n + i];
        const double dd = d.x * d.x + d.y * d.y;
        B[e] = cmul(B[e], make_double2(d.x / dd, -d.y / dd));
    }
}

unsigned grid_for(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kThreads - 1) / kThreads, 8192));
}

// Solve A X = B in place (A: n x n, B: n x m, row-major); false if a pivot
// vanishes or is not finite.
bool lu_solve(kgf_ctx* ctx, double2* A, int n, double2* B, int m, double* piv_dev) {
    for (int k = 0; k < n; ++k) {
        {
            Prof pr(ctx, "k_lu_pivot");
            hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(256), 0, ctx->stream, A, n, B, m, k, piv_dev);
            check_launch("k_lu_pivot");
        }
        const int64_t total = (int64_t)(n - k - 1) * ((n - k - 1) + m);
        if (total > 0) {
            Prof pr(ctx, "k_lu_elim");
            hipLaunchKernelGGL(k_lu_elim, dim3(grid_for(total)), dim3(kThreads), 0, ctx->stream, A, n, B, m, k);
            check_launch("k_lu_elim");
        }
    }
    std::vector<double> piv(n);
    KGF_HIP(hipMemcpyAsync(piv.data(), piv_dev, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    for (int k = 0; k < n; ++k)
        if (!(piv[k] > 0.0) || !std::isfinite(piv[k])) return false;
    for (int k = n - 1; k > 0; --k) {
        const int64_t total = (int64_t)k * m;
        Prof pr(ctx, "k_lu_back");
        hipLaunchKernelGGL(k_lu_back, dim3(grid_for(total)), dim3(kThreads), 0, ctx->stream, A, n, B, m, k);
        check_launch("k_lu_back");
    }
    hipLaunchKernelGGL(k_lu_scale, dim3(grid_for((int64_t)n * m)), dim3(kThreads), 0, ctx->stream, A, n, B, m);
    check_launch("k_lu_scale");
    return true;
}

// G[a][b][i][j] = Gc[a][b][i][j] + C[(i N + p) * ldc + j N + q] with
// (p, q) = (a forward, b backward) for G^< and (a backward, b forward) for G^>
// (N = 2 nt + ntau contour points; backward point of t_b: 2 nt - 1 - b)
__global__ void k_extract(const double2* __restrict__ Gcl, const double2* __restrict__ Gcg,
                          const double2* __restrict__ C, int64_t ldc, int nt, int ntau, int nc,
                          double2* __restrict__ Gl, double2* __restrict__ Gg) {
    const int N = 2 * nt + ntau;
    const int64_t total = (int64_t)nt * nt * nc * nc;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % nc);
        const int i = (int)((e / nc) % nc);
        const int b = (int)((e / ((int64_t)nc * nc)) % nt);
        const int a = (int)(e / ((int64_t)nc * nc * nt));
        const double2 cl = C[((int64_t)i * N + a) * ldc + (int64_t)j * N + (2 * nt - 1 - b)];
        const double2 cg = C[((int64_t)i * N + (2 * nt - 1 - a)) * ldc + (int64_t)j * N + b];
        Gl[e] = make_double2(Gcl[e].x + cl.x, Gcl[e].y + cl.y);
        Gg[e] = make_double2(Gcg[e].x + cg.x, Gcg[e].y + cg.y);
    }
}

// the mixed components: Gmx[a][jt][i][j] (forward t_a, imaginary tau_jt) and
// Gmxl[jt][b][i][j] (imaginary tau_jt, forward t_b); either output may be null
__global__ void k_extract_mixed(const double2* __restrict__ Gcmx, const double2* __restrict__ Gcmxl,
                                const double2* __restrict__ C, int64_t ldc, int nt, int ntau, int nc,
                                double2* __restrict__ Gmx, double2* __restrict__ Gmxl) {
    const int N = 2 * nt + ntau;
    const int64_t total = (int64_t)nt * ntau * nc * nc;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % nc);
        const int i = (int)((e / nc) % nc);
        const int64_t r = e / ((int64_t)nc * nc);
        if (Gmx) {   // e indexes [a][jt][i][j]
            const int jt = (int)(r % ntau), a = (int)(r / ntau);
            const double2 c = C[((int64_t)i * N + a) * ldc + (int64_t)j * N + 2 * nt + jt];
            Gmx[e] = make_double2(Gcmx[e].x + c.x, Gcmx[e].y + c.y);
        }
        if (Gmxl) {  // e indexes [jt][b][i][j]
            const int b = (int)(r % nt), jt = (int)(r / nt);
            const double2 c = C[((int64_t)i * N + 2 * nt + jt) * ldc + (int64_t)j * N + b];
            Gmxl[e] = make_double2(Gcmxl[e].x + c.x, Gcmxl[e].y + c.y);
        }
    }
}

// Eqs. (gb1), (gb2) for site 1 of an L_b-site chain with hopping -T_b between
// neighbours: levels e_k = -2 T_b cos(k pi / (L_b + 1)), weights
// u_k^2 = 2 sin^2(k pi / (L_b + 1)) / (L_b + 1), occupations 1 / (e^{beta e} + 1)
// (beta = inf: 1, 1/2, 0 for e <, =, > 0, |e| <= 1e-12 max(1, 2|T_b|) counting as
// zero); one thread per time difference d = a - b.
__global__ void k_bath_chain(int Lb, double Tb, double beta, int nt, double dt, double2* __restrict__ gl_d,
                             double2* __restrict__ gg_d) {
    const int nd = 2 * nt - 1;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nd; e += gridDim.x * blockDim.x) {
        const double tau = (double)(e - (nt - 1)) * dt;
        double lr = 0.0, li = 0.0, gr = 0.0, gi = 0.0;
        for (int k = 1; k <= Lb; ++k) {
            const double th = M_PI * k / (Lb + 1);
            const double ek = -2.0 * Tb * cos(th);
            const double sn = sin(th);
            const double u2 = 2.0 * sn * sn / (Lb + 1);
            const bool zero = fabs(ek) <= 1e-12 * fmax(1.0, 2.0 * fabs(Tb));   // a zero level, up to rounding
            double f;
            if (isinf(beta))
                f = zero ? 0.5 : (ek < 0.0 ? 1.0 : 0.0);
            else
                f = 1.0 / (exp(beta * ek) + 1.0);
            double s, c;
            sincos(ek * tau, &s, &c);        // e^{-i e tau} = c - i s
            // G^< = +i u2 f (c - i s) = u2 f (s + i c);  G^> = -i u2 (1-f) (c - i s) = u2 (1-f) (-s - i c)
            lr += u2 * f * s;
            li += u2 * f * c;
            gr -= u2 * (1.0 - f) * s;
            gi -= u2 * (1.0 - f) * c;
        }
        gl_d[e] = make_double2(lr, li);
        gg_d[e] = make_double2(gr, gi);
    }
}

__global__ void k_expand_diff(const double2* __restrict__ gl_d, const double2* __restrict__ gg_d, int nt,
                              double2* __restrict__ Gl, double2* __restrict__ Gg) {
    const int64_t total = (int64_t)nt * nt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e / nt), b = (int)(e % nt);
        Gl[e] = gl_d[a - b + nt - 1];
        Gg[e] = gg_d[a - b + nt - 1];
    }
}

// f(e) e^{e x} and (1 - f(e)) e^{-e x} for 0 <= x <= beta without overflow
// (beta = inf: occupation 1, 1/2, 0 for a negative, zero, positive level)
__device__ __forceinline__ double fermi_exp(double e, double x, double beta, bool zero) {
    if (isinf(beta)) return zero ? 0.5 : (e < 0.0 ? exp(e * x) : 0.0);
    if (e <= 0.0) return exp(e * x) / (exp(beta * e) + 1.0);
    return exp(-e * (beta - x)) / (1.0 + exp(-beta * e));
}
__device__ __forceinline__ double hole_exp(double e, double x, double beta, bool zero) {
    return fermi_exp(-e, x, beta, zero);
}

// Eqs. (gb1), (gb2) on complex contour times for site 1 of the chain (levels
// and weights as k_bath_chain): mixed [a][j] = i sum u2 f e^{e tau_j} e^{-i e t_a},
// mixed_left [j][b] = -i sum u2 (1-f) e^{-e tau_j} e^{+i e t_b},
// vertical [d]: G^> = -i sum u2 (1-f) e^{-e tau_d}, G^< = i sum u2 f e^{e tau_d}.
// One thread per (a, j) of the nt x ntau mesh (a < nt also writes mixed_left
// [j][a]); threads with a == nt write the vertical functions at d = j.
__global__ void k_bath_chain_tau(int Lb, double Tb, double beta, int nt, double dt, int ntau, double dtau,
                                 double2* __restrict__ mx, double2* __restrict__ mxl, double2* __restrict__ vg,
                                 double2* __restrict__ vl) {
    const int64_t total = (int64_t)(nt + 1) * ntau;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e / ntau), j = (int)(e % ntau);
        const double tau = j * dtau;
        double mr = 0.0, mi = 0.0, xr = 0.0, xi = 0.0;   // mixed, mixed_left (or vertical G^>, G^<)
        for (int k = 1; k <= Lb; ++k) {
            const double th = M_PI * k / (Lb + 1);
            const double ek = -2.0 * Tb * cos(th);
            const double sn = sin(th);
            const double u2 = 2.0 * sn * sn / (Lb + 1);
            const bool zero = fabs(ek) <= 1e-12 * fmax(1.0, 2.0 * fabs(Tb));
            const double fe = u2 * fermi_exp(ek, tau, beta, zero);
            const double he = u2 * hole_exp(ek, tau, beta, zero);
            if (a < nt) {
                double sa, ca;
                sincos(ek * a * dt, &sa, &ca);   // e^{-i e t} = ca - i sa
                // i fe (ca - i sa) = fe (sa + i ca);  -i he (ca + i sa) = he (sa - i ca)
                mr += fe * sa;
                mi += fe * ca;
                xr += he * sa;
                xi -= he * ca;
            } else {
                xi -= he;   // vertical G^>: -i he
                mi += fe;   // vertical G^<: +i fe
            }
        }
        if (a < nt) {
            mx[(int64_t)a * ntau + j] = make_double2(mr, mi);
            mxl[(int64_t)j * nt + a] = make_double2(xr, xi);
        } else {
            vg[j] = make_double2(0.0, xi);
            vl[j] = make_double2(0.0, mi);
        }
    }
}

// The cluster block of the CPT equation on the contour of nt real and ntau
// imaginary mesh points (ntau = 0: the Keldysh contour alone), bath
// eliminated; see the file comment.  Gc: the cluster's components
// [..][n_c][n_c]; Gb: the bath's site-1 components.  Outputs G^<, G^>
// [nt][nt][n_c][n_c] and, when given, the mixed components.
struct CompPtrs {
    const double2 *l, *g, *mx, *mxl, *vg, *vl;
};

void necpt_solve(kgf_ctx* ctx, int nt, int ntau, int n_c, int boundary, double dt, double dtau, double V,
                 const CompPtrs& gc, const CompPtrs& gb, double2* G_lesser, double2* G_greater, double2* G_mixed,
                 double2* G_mixed_left) {
    const int n = 2 * nt + ntau, m = n * n_c;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    ensure_device_fits(sizeof(double2) * (3 * nn + 3 * nm + (size_t)m * m), "NE-CPT contour matrices");
    auto buf = [&](const char* name, size_t elems) {
        return static_cast<double2*>(workspace(ctx, name, sizeof(double2) * elems));
    };
    double2* P = buf("cpt_P", nn);     // G^c_bb on the contour
    double2* K = buf("cpt_K", nn);     // w Sigma w
    double2* A = buf("cpt_A", nn);     // 1 - P K
    double2* X = buf("cpt_X", nm);     // G^c_bj -> X_j (columns j n + q)
    double2* Y = buf("cpt_Y", nm);     // K X
    double2* R = buf("cpt_R", nm);     // G^c_ib stacked by rows (i n + p)
    double2* C = buf("cpt_C", (size_t)m * m);
    double* piv = static_cast<double*>(workspace(ctx, "cpt_piv", sizeof(double) * n));
    const int64_t q2 = (int64_t)n_c * n_c;
    auto cluster = [&](int i, int j) {   // orbital pair (i, j) of the cluster components
        const int64_t o = (int64_t)i * n_c + j;
        CFn f;
        f.l = gc.l + o;
        f.g = gc.g + o;
        f.mx = gc.mx ? gc.mx + o : nullptr;
        f.mxl = gc.mxl ? gc.mxl + o : nullptr;
        f.vg = gc.vg ? gc.vg + o : nullptr;
        f.vl = gc.vl ? gc.vl + o : nullptr;
        f.la = (int64_t)nt * q2;
        f.lb = q2;
        f.ma = (int64_t)ntau * q2;
        f.mj = q2;
        f.xj = (int64_t)nt * q2;
        f.xb = q2;
        f.vd = q2;
        return f;
    };
    CFn fb;
    fb.l = gb.l;
    fb.g = gb.g;
    fb.mx = gb.mx;
    fb.mxl = gb.mxl;
    fb.vg = gb.vg;
    fb.vl = gb.vl;
    fb.la = nt;
    fb.lb = 1;
    fb.ma = ntau;
    fb.mj = 1;
    fb.xj = nt;
    fb.xb = 1;
    fb.vd = 1;
    const unsigned g = grid_for((int64_t)nn);
    auto contour = [&](const CFn& f, double s, int wts, int rhs, double2* out, int64_t ldo) {
        hipLaunchKernelGGL(k_to_contour, dim3(g), dim3(kThreads), 0, ctx->stream, f, nt, ntau, s, wts, rhs, dt, dtau,
                           out, ldo);
        check_launch("k_to_contour");
    };
    // kernels of the integral (P, K, R): row values; right-hand sides (X): rhs values
    contour(cluster(boundary, boundary), 1.0, 0, 0, P, n);
    contour(fb, V * V, 1, 0, K, n);
    for (int j = 0; j < n_c; ++j) {
        contour(cluster(boundary, j), 1.0, 0, 1, X + (size_t)j * n, m);
        contour(cluster(j, boundary), 1.0, 0, 0, R + (size_t)j * nn, n);
    }
    hipLaunchKernelGGL(k_identity, dim3(g), dim3(kThreads), 0, ctx->stream, A, n);
    check_launch("k_identity");
    zgemm(ctx, n, n, n, make_double2(-1.0, 0.0), P, n, K, n, make_double2(1.0, 0.0), A, n);
    KGF_REQUIRE(lu_solve(ctx, A, n, X, m, piv), KGF_EINVAL, "NE-CPT: singular contour matrix 1 - G^c_bb K");
    zgemm(ctx, n, m, n, make_double2(1.0, 0.0), K, n, X, m, make_double2(0.0, 0.0), Y, m);
    zgemm(ctx, m, m, n, make_double2(1.0, 0.0), R, n, Y, m, make_double2(0.0, 0.0), C, m);
    hipLaunchKernelGGL(k_extract, dim3(grid_for((int64_t)nt * nt * n_c * n_c)), dim3(kThreads), 0, ctx->stream,
                       gc.l, gc.g, C, (int64_t)m, nt, ntau, n_c, G_lesser, G_greater);
    check_launch("k_extract");
    if (ntau > 0 && (G_mixed || G_mixed_left)) {
        hipLaunchKernelGGL(k_extract_mixed, dim3(grid_for((int64_t)nt * ntau * n_c * n_c)), dim3(kThreads), 0,
                           ctx->stream, gc.mx, gc.mxl, C, (int64_t)m, nt, ntau, n_c, G_mixed, G_mixed_left);
        check_launch("k_extract_mixed");
    }
    sync(ctx);
}

}  // namespace

}  // namespace kgf

using namespace kgf;

extern "C" int kgf_bath_chain(kgf_ctx* ctx, int L_b, double T_b, double beta, int nt, double dt,
                              kgf_c128* G_lesser, kgf_c128* G_greater) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && G_lesser && G_greater, KGF_EINVAL, "kgf_bath_chain: NULL argument");
        KGF_REQUIRE(L_b >= 1 && nt >= 1 && std::isfinite(T_b) && std::isfinite(dt) && dt >= 0.0 &&
                        !std::isnan(beta) && beta > 0.0,
                    KGF_EINVAL, "kgf_bath_chain: bad L_b / nt / T_b / dt / beta");
        KGF_HIP(hipSetDevice(ctx->device));
        const int nd = 2 * nt - 1;
        double2* d = static_cast<double2*>(workspace(ctx, "cpt_bath_d", sizeof(double2) * 2 * (size_t)nd));
        hipLaunchKernelGGL(k_bath_chain, dim3((unsigned)((nd + 63) / 64)), dim3(64), 0, ctx->stream, L_b, T_b, beta,
                           nt, dt, d, d + nd);
        check_launch("k_bath_chain");
        hipLaunchKernelGGL(k_expand_diff, dim3(grid_for((int64_t)nt * nt)), dim3(kThreads), 0, ctx->stream, d,
                           d + nd, nt, reinterpret_cast<double2*>(G_lesser), reinterpret_cast<double2*>(G_greater));
        check_launch("k_expand_diff");
        sync(ctx);
    });
}

extern "C" int kgf_necpt(kgf_ctx* ctx, int nt, int n_c, int boundary, double dt, double V,
                         const kgf_c128* Gc_lesser, const kgf_c128* Gc_greater, const kgf_c128* Gb_lesser,
                         const kgf_c128* Gb_greater, kgf_c128* G_lesser, kgf_c128* G_greater) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && Gc_lesser && Gc_greater && Gb_lesser && Gb_greater && G_lesser && G_greater, KGF_EINVAL,
                    "kgf_necpt: NULL argument");
        KGF_REQUIRE(nt >= 1 && n_c >= 1 && boundary >= 0 && boundary < n_c, KGF_EINVAL,
                    "kgf_necpt: bad nt / n_c / boundary");
        KGF_REQUIRE(std::isfinite(dt) && dt >= 0.0 && std::isfinite(V), KGF_EINVAL, "kgf_necpt: bad dt / V");
        KGF_REQUIRE((int64_t)2 * nt * n_c <= 65536, KGF_EUNSUPPORTED, "kgf_necpt: 2 nt n_c above 65536");
        KGF_HIP(hipSetDevice(ctx->device));
        CompPtrs gc{reinterpret_cast<const double2*>(Gc_lesser), reinterpret_cast<const double2*>(Gc_greater),
                    nullptr, nullptr, nullptr, nullptr};
        CompPtrs gb{reinterpret_cast<const double2*>(Gb_lesser), reinterpret_cast<const double2*>(Gb_greater),
                    nullptr, nullptr, nullptr, nullptr};
        necpt_solve(ctx, nt, 0, n_c, boundary, dt, 0.0, V, gc, gb, reinterpret_cast<double2*>(G_lesser),
                    reinterpret_cast<double2*>(G_greater), nullptr, nullptr);
        progress(ctx, "necpt", 1, 1);
    });
}

static bool contour_fn_complete(const kgf_contour_fn* f) {
    return f && f->lesser && f->greater && f->mixed && f->mixed_left && f->vert_greater && f->vert_lesser;
}

static CompPtrs comp_ptrs(const kgf_contour_fn* f) {
    return CompPtrs{reinterpret_cast<const double2*>(f->lesser), reinterpret_cast<const double2*>(f->greater),
                    reinterpret_cast<const double2*>(f->mixed), reinterpret_cast<const double2*>(f->mixed_left),
                    reinterpret_cast<const double2*>(f->vert_greater), reinterpret_cast<const double2*>(f->vert_lesser)};
}

extern "C" int kgf_bath_chain_contour(kgf_ctx* ctx, int L_b, double T_b, double beta, int nt, double dt, int ntau,
                                      double dtau, const kgf_contour_fn* out) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && contour_fn_complete(out), KGF_EINVAL, "kgf_bath_chain_contour: NULL argument");
        KGF_REQUIRE(L_b >= 1 && nt >= 1 && ntau >= 1 && std::isfinite(T_b) && std::isfinite(dt) && dt >= 0.0 &&
                        std::isfinite(dtau) && dtau >= 0.0 && !std::isnan(beta) && beta > 0.0 &&
                        (std::isinf(beta) || (ntau - 1) * dtau <= beta * (1.0 + 1e-12)),
                    KGF_EINVAL, "kgf_bath_chain_contour: bad L_b / nt / ntau / T_b / dt / dtau / beta");
        KGF_HIP(hipSetDevice(ctx->device));
        const int nd = 2 * nt - 1;
        double2* d = static_cast<double2*>(workspace(ctx, "cpt_bath_d", sizeof(double2) * 2 * (size_t)nd));
        hipLaunchKernelGGL(k_bath_chain, dim3((unsigned)((nd + 63) / 64)), dim3(64), 0, ctx->stream, L_b, T_b, beta,
                           nt, dt, d, d + nd);
        check_launch("k_bath_chain");
        hipLaunchKernelGGL(k_expand_diff, dim3(grid_for((int64_t)nt * nt)), dim3(kThreads), 0, ctx->stream, d,
                           d + nd, nt, reinterpret_cast<double2*>(out->lesser), reinterpret_cast<double2*>(out->greater));
        check_launch("k_expand_diff");
        const int64_t tot = (int64_t)(nt + 1) * ntau;
        hipLaunchKernelGGL(k_bath_chain_tau, dim3(grid_for(tot)), dim3(kThreads), 0, ctx->stream, L_b, T_b, beta, nt,
                           dt, ntau, dtau, reinterpret_cast<double2*>(out->mixed),
                           reinterpret_cast<double2*>(out->mixed_left), reinterpret_cast<double2*>(out->vert_greater),
                           reinterpret_cast<double2*>(out->vert_lesser));
        check_launch("k_bath_chain_tau");
        sync(ctx);
    });
}

// A cluster's contour function from the four-step outputs (orbitals
// selected by sel), optionally completed for a finite imaginary branch.
struct ClusterIn {
    const double2* gl;
    const double2* gg;
    const double2* gm;     // [2][ntau][no][no]
    const double2* mx;     // [nt][ntau][no][no]
    const double2* mxl;    // [ntau][nt][no][no]
};
struct ClusterOut {
    double2* gl;
    double2* gg;
    double2* mx;
    double2* mxl;
    double2* vg;
    double2* vl;
};

__device__ __forceinline__ double2 times_i(double2 z) { return make_double2(-z.y, z.x); }

__global__ void k_cluster_contour(int nt, int ntau, int no, const int* __restrict__ sel, int nc, int kms,
                                  ClusterIn in, ClusterOut out) {
    const int64_t q = (int64_t)nc * nc;
    const int64_t n_gl = (int64_t)nt * nt * q, n_mx = (int64_t)nt * ntau * q, n_v = (int64_t)ntau * q;
    const int64_t total = 2 * n_gl + 2 * n_mx + 2 * n_v;
    auto at = [&](int64_t outer, int a, int b) -> int64_t { return outer * no * no + (int64_t)sel[a] * no + sel[b]; };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        // output array and element index within it
        int64_t r = i;
        int which;
        if (r < n_gl) which = 0;
        else if ((r -= n_gl) < n_gl) which = 1;
        else if ((r -= n_gl) < n_mx) which = 2;
        else if ((r -= n_mx) < n_mx) which = 3;
        else if ((r -= n_mx) < n_v) which = 4;
        else {
            r -= n_v;
            which = 5;
        }
        const int a = (int)((r / nc) % nc), b = (int)(r % nc);
        const int64_t outer = r / q;
        if (which <= 1) {
            (which == 0 ? out.gl : out.gg)[r] = (which == 0 ? in.gl : in.gg)[at(outer, a, b)];
        } else if (which == 2) {                       // G^|(t, tau): outer = t * ntau + j
            const int t = (int)(outer / ntau), j = (int)(outer % ntau);
            double2 v = in.mx[at(outer, a, b)];
            if (kms) {
                const double2 w = in.mxl[at((int64_t)(ntau - 1 - j) * nt + t, b, a)];
                v.x += w.x;
                v.y -= w.y;
            }
            out.mx[r] = v;
        } else if (which == 3) {                       // G^|(tau, t): outer = j * nt + t
            const int j = (int)(outer / nt), t = (int)(outer % nt);
            double2 v = in.mxl[at(outer, a, b)];
            if (kms) {
                const double2 w = in.mx[at((int64_t)t * ntau + (ntau - 1 - j), b, a)];
                v.x += w.x;
                v.y -= w.y;
            }
            out.mxl[r] = v;
        } else {                                       // vertical: outer = j
            const int j = (int)outer;
            const double2* g0 = in.gm + (which == 4 ? 0 : (int64_t)ntau * no * no);   // +tau (4) or -tau (5)
            const double2* g1 = in.gm + (which == 4 ? (int64_t)ntau * no * no : 0);
            double2 v = times_i(g0[at(j, a, b)]);
            if (kms) {
                const double2 w = times_i(g1[at(ntau - 1 - j, a, b)]);
                v.x -= w.x;
                v.y -= w.y;
            }
            (which == 4 ? out.vg : out.vl)[r] = v;
        }
    }
}

extern "C" int kgf_cluster_contour(kgf_ctx* ctx, int nt, int ntau, int n_orb, const kgf_c128* host_G_lesser,
                                   const kgf_c128* host_G_greater, const kgf_c128* host_G_matsubara,
                                   const kgf_c128* host_G_mixed, const kgf_c128* host_G_mixed_left,
                                   const int* host_sel, int n_c, int kms, const kgf_contour_fn* out) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && host_G_lesser && host_G_greater && host_G_matsubara && host_G_mixed && host_G_mixed_left &&
                        contour_fn_complete(out),
                    KGF_EINVAL, "kgf_cluster_contour: NULL argument");
        KGF_REQUIRE(nt >= 1 && ntau >= 2 && n_orb >= 1 && n_c >= 1 && (host_sel || n_c == n_orb) &&
                        (kms == 0 || kms == 1),
                    KGF_EINVAL, "kgf_cluster_contour: bad nt / ntau / n_orb / n_c / kms");
        std::vector<int> sel((size_t)n_c);
        for (int a = 0; a < n_c; ++a) {
            sel[a] = host_sel ? host_sel[a] : a;
            KGF_REQUIRE(sel[a] >= 0 && sel[a] < n_orb, KGF_EINVAL, "kgf_cluster_contour: orbital index out of range");
        }
        KGF_HIP(hipSetDevice(ctx->device));
        const size_t oo = (size_t)n_orb * n_orb;
        const size_t b_gl = sizeof(double2) * (size_t)nt * nt * oo, b_gm = sizeof(double2) * 2 * (size_t)ntau * oo,
                     b_mx = sizeof(double2) * (size_t)nt * ntau * oo;
        char* w = static_cast<char*>(workspace(ctx, "cpt_cluster_in", 2 * b_gl + b_gm + 2 * b_mx + sizeof(int) * n_c));
        ClusterIn in;
        in.gl = reinterpret_cast<const double2*>(w);
        in.gg = reinterpret_cast<const double2*>(w + b_gl);
        in.gm = reinterpret_cast<const double2*>(w + 2 * b_gl);
        in.mx = reinterpret_cast<const double2*>(w + 2 * b_gl + b_gm);
        in.mxl = reinterpret_cast<const double2*>(w + 2 * b_gl + b_gm + b_mx);
        int* dsel = reinterpret_cast<int*>(w + 2 * b_gl + b_gm + 2 * b_mx);
        KGF_HIP(hipMemcpyAsync(w, host_G_lesser, b_gl, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(w + b_gl, host_G_greater, b_gl, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(w + 2 * b_gl, host_G_matsubara, b_gm, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(w + 2 * b_gl + b_gm, host_G_mixed, b_mx, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(w + 2 * b_gl + b_gm + b_mx, host_G_mixed_left, b_mx, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(dsel, sel.data(), sizeof(int) * n_c, hipMemcpyHostToDevice, ctx->stream));
        ClusterOut o{reinterpret_cast<double2*>(out->lesser), reinterpret_cast<double2*>(out->greater),
                     reinterpret_cast<double2*>(out->mixed), reinterpret_cast<double2*>(out->mixed_left),
                     reinterpret_cast<double2*>(out->vert_greater), reinterpret_cast<double2*>(out->vert_lesser)};
        const int64_t total = (int64_t)n_c * n_c * (2 * (int64_t)nt * nt + 2 * (int64_t)nt * ntau + 2 * (int64_t)ntau);
        hipLaunchKernelGGL(k_cluster_contour, dim3(grid_for(total)), dim3(kThreads), 0, ctx->stream, nt, ntau, n_orb,
                           dsel, n_c, kms, in, o);
        check_launch("k_cluster_contour");
        sync(ctx);   // the host arrays may go away on return
    });
}

extern "C" int kgf_necpt_contour(kgf_ctx* ctx, int nt, int ntau, int n_c, int boundary, double dt, double dtau,
                                 double V, const kgf_contour_fn* Gc, const kgf_contour_fn* Gb, kgf_c128* G_lesser,
                                 kgf_c128* G_greater, kgf_c128* G_mixed, kgf_c128* G_mixed_left) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && contour_fn_complete(Gc) && contour_fn_complete(Gb) && G_lesser && G_greater, KGF_EINVAL,
                    "kgf_necpt_contour: NULL argument");
        KGF_REQUIRE(nt >= 1 && ntau >= 2 && n_c >= 1 && boundary >= 0 && boundary < n_c, KGF_EINVAL,
                    "kgf_necpt_contour: bad nt / ntau / n_c / boundary");
        KGF_REQUIRE(std::isfinite(dt) && dt >= 0.0 && std::isfinite(dtau) && dtau > 0.0 && std::isfinite(V),
                    KGF_EINVAL, "kgf_necpt_contour: bad dt / dtau / V");
        KGF_REQUIRE((int64_t)(2 * nt + ntau) * n_c <= 65536, KGF_EUNSUPPORTED,
                    "kgf_necpt_contour: (2 nt + ntau) n_c above 65536");
        KGF_HIP(hipSetDevice(ctx->device));
        necpt_solve(ctx, nt, ntau, n_c, boundary, dt, dtau, V, comp_ptrs(Gc), comp_ptrs(Gb),
                    reinterpret_cast<double2*>(G_lesser), reinterpret_cast<double2*>(G_greater),
                    reinterpret_cast<double2*>(G_mixed), reinterpret_cast<double2*>(G_mixed_left));
        progress(ctx, "necpt", 1, 1);
    });
}
