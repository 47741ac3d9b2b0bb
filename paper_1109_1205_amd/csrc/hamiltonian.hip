// Matrix-free H.v in one (N_up, N_dn) sector and the ladder operators.
//
// With a state stored as the D_up x D_dn row-major matrix V[u, d], the
// Hamiltonian of Sec. 3 / Sec. 4 separates into
//     (H V)[u, d] = sum_u' T_up[u, u'] V[u', d]        (up-spin hops)
//                 + sum_d' T_dn[d, d'] V[u, d']        (down-spin hops)
//                 + diag(u, d) V[u, d],
//     diag(u, d)  = e_up[u] + e_dn[d] + sum_i U_i bit_i(m_u & m_d),
// where T_sigma is the single-species hopping matrix (ELL table built in
// basis.hip).  One block computes one output row u: the up-spin hops read
// whole rows V[u', :] (coalesced along d), the down-spin hops gather inside
// row u (L1/L2 resident), the diagonal is evaluated on the fly from the two
// masks.  H.v is sparse and memory bound: no matrix cores are involved.
#include "kgf_internal.h"

namespace kgf {

namespace {

struct HvTables {
    int64_t Dup, Ddn;
    const uint32_t* mu;
    const uint32_t* md;
    const int32_t* cnt_up;
    const uint32_t* ent_up;
    const int32_t* cnt_dn;
    const uint32_t* ent_dn;
    const double* eu;     // on-site energy of each up mask (eps_up)
    const double* ed;     // on-site energy of each down mask (eps_dn)
    const double* t;      // [nb]
    const double* Utab;   // [3 * 256]
    double U0;
    int nb;
};

HvTables make_tables(kgf_model* model, const kgf_sector* sec) {
    HopTable& tu = hop_table(model, sec->n_up);
    HopTable& td = hop_table(model, sec->n_dn);
    HvTables T;
    T.Dup = sec->d_up;
    T.Ddn = sec->d_dn;
    T.mu = tu.masks.as<uint32_t>();
    T.md = td.masks.as<uint32_t>();
    T.cnt_up = tu.count.as<int32_t>();
    T.ent_up = tu.ent.as<uint32_t>();
    T.cnt_dn = td.count.as<int32_t>();
    T.ent_dn = td.ent.as<uint32_t>();
    T.eu = tu.e_up.as<double>();
    T.ed = td.e_dn.as<double>();
    T.t = model->d_t.as<double>();
    T.Utab = model->d_Utab.as<double>();
    T.U0 = model->U.empty() ? 0.0 : model->U[0];
    T.nb = model->nb;
    return T;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// sum over the block in a fixed order; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

// MODE 0: y = H x.
// MODE 1: y = s * H x - bp * xp, part = Re <s x, y>   (one Lanczos step)
template <int MODE, bool UNIFORM_U>
__global__ __launch_bounds__(kThreads) void k_hv(HvTables T, const double2* __restrict__ X,
                                                 int64_t x_col, const double2* __restrict__ XP,
                                                 int64_t xp_col, double2* __restrict__ Y,
                                                 int64_t y_col, const double* __restrict__ s_k,
                                                 const double* __restrict__ b_k,
                                                 const double* __restrict__ s_km1, int stride,
                                                 double* __restrict__ part) {
    __shared__ double s_negt[kMaxBonds + 1];
    __shared__ double s_U[UNIFORM_U ? 1 : 3 * 256];
    __shared__ double s_upval[kMaxBonds + 1];
    __shared__ int64_t s_uprow[kMaxBonds + 1];
    __shared__ double s_red[kThreads / 64];

    const int64_t u = blockIdx.x;
    const int c = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t Ddn = T.Ddn;
    const double2* __restrict__ x = X + c * x_col;
    double2* __restrict__ y = Y + c * y_col;

    for (int b = tid; b < T.nb; b += blockDim.x) s_negt[b] = -T.t[b];
    if (!UNIFORM_U)
        for (int i = tid; i < 3 * 256; i += blockDim.x) s_U[i] = T.Utab[i];
    __syncthreads();
    const int cu = T.cnt_up[u];
    for (int k = tid; k < cu; k += blockDim.x) {
        uint32_t e = T.ent_up[(int64_t)k * T.Dup + u];
        double v = s_negt[(e >> 24) & 127u];
        s_upval[k] = (e >> 31) ? -v : v;
        s_uprow[k] = (int64_t)(e & 0xFFFFFFu) * Ddn;
    }
    __syncthreads();

    double sc = 1.0, bp = 0.0;
    if (MODE == 1) {
        sc = s_k[c * stride];
        if (XP) bp = b_k[c * stride] * s_km1[c * stride];
    }
    const uint32_t mu = T.mu[u];
    const double eu = T.eu[u];
    const double2* __restrict__ xrow = x + u * Ddn;
    double dot = 0.0;

    for (int64_t d = tid; d < Ddn; d += blockDim.x) {
        const double2 xv = xrow[d];
        const uint32_t both = mu & T.md[d];
        double dg = eu + T.ed[d];
        if (UNIFORM_U) {
            dg += T.U0 * (double)__popc(both);
        } else {
            dg += s_U[both & 255u] + s_U[256 + ((both >> 8) & 255u)] + s_U[512 + ((both >> 16) & 255u)];
        }
        double ar = dg * xv.x, ai = dg * xv.y;
        for (int k = 0; k < cu; ++k) {
            const double2 z = x[s_uprow[k] + d];
            const double tv = s_upval[k];
            ar = fma(tv, z.x, ar);
            ai = fma(tv, z.y, ai);
        }
        const int cd = T.cnt_dn[d];
        for (int k = 0; k < cd; ++k) {
            const uint32_t e = T.ent_dn[(int64_t)k * Ddn + d];
            double tv = s_negt[(e >> 24) & 127u];
            tv = (e >> 31) ? -tv : tv;
            const double2 z = xrow[e & 0xFFFFFFu];
            ar = fma(tv, z.x, ar);
            ai = fma(tv, z.y, ai);
        }
        double2 out;
        if (MODE == 0) {
            out.x = ar;
            out.y = ai;
        } else {
            out.x = sc * ar;
            out.y = sc * ai;
            if (bp != 0.0) {
                const double2 p = (XP + c * xp_col)[u * Ddn + d];
                out.x = fma(-bp, p.x, out.x);
                out.y = fma(-bp, p.y, out.y);
            }
            dot = fma(sc * xv.x, out.x, dot);
            dot = fma(sc * xv.y, out.y, dot);
        }
        y[u * Ddn + d] = out;
    }
    if (MODE == 1) {
        double s = block_sum(dot, s_red);
        if (tid == 0) part[(int64_t)c * gridDim.x + u] = s;
    }
}

// Row-in-LDS variant: the block stages its input row x[u, :] in LDS, so the
// down-spin gathers (random inside the row) are served by LDS; only the
// up-spin row reads go to the memory hierarchy.  Blocks are mapped to the
// 8 XCDs so that each XCD walks a contiguous range of rows (block b runs on
// XCD b mod 8): most up-spin hops connect rows less than a few hundred
// apart, so their source rows stay in that XCD's L2.
constexpr int kHvThreads = 1024;
constexpr size_t kRowLdsMax = 78 * 1024;

template <int MODE, bool UNIFORM_U>
__global__ __launch_bounds__(kHvThreads) void k_hv_lds(HvTables T, int rows_per_xcd,
                                                       const double2* __restrict__ X, int64_t x_col,
                                                       const double2* __restrict__ XP, int64_t xp_col,
                                                       double2* __restrict__ Y, int64_t y_col,
                                                       const double* __restrict__ s_k,
                                                       const double* __restrict__ b_k,
                                                       const double* __restrict__ s_km1, int stride,
                                                       double* __restrict__ part) {
    extern __shared__ double2 srow[];
    __shared__ double s_negt[kMaxBonds + 1];
    __shared__ double s_U[UNIFORM_U ? 1 : 3 * 256];
    __shared__ double s_upval[kMaxBonds + 1];
    __shared__ int64_t s_uprow[kMaxBonds + 1];
    __shared__ double s_red[kHvThreads / 64];

    const int blk = blockIdx.x;
    const int64_t u = (int64_t)(blk & 7) * rows_per_xcd + (blk >> 3);
    if (u >= T.Dup) return;   // uniform over the block
    const int c = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t Ddn = T.Ddn;
    const double2* __restrict__ x = X + c * x_col;
    double2* __restrict__ y = Y + c * y_col;
    const double2* __restrict__ xrow = x + u * Ddn;

    for (int64_t d = tid; d < Ddn; d += blockDim.x) srow[d] = xrow[d];
    for (int b = tid; b < T.nb; b += blockDim.x) s_negt[b] = -T.t[b];
    if (!UNIFORM_U)
        for (int i = tid; i < 3 * 256; i += blockDim.x) s_U[i] = T.Utab[i];
    __syncthreads();
    const int cu = T.cnt_up[u];
    for (int k = tid; k < cu; k += blockDim.x) {
        uint32_t e = T.ent_up[(int64_t)k * T.Dup + u];
        double v = s_negt[(e >> 24) & 127u];
        s_upval[k] = (e >> 31) ? -v : v;
        s_uprow[k] = (int64_t)(e & 0xFFFFFFu) * Ddn;
    }
    __syncthreads();

    double sc = 1.0, bp = 0.0;
    if (MODE == 1) {
        sc = s_k[c * stride];
        if (XP) bp = b_k[c * stride] * s_km1[c * stride];
    }
    const uint32_t mu = T.mu[u];
    const double eu = T.eu[u];
    double dot = 0.0;
    // Gathers are issued in predicated batches of kBatch so that many loads
    // are in flight per thread (the hop counts are data dependent).
    constexpr int kBatch = 8;
    for (int64_t d = tid; d < Ddn; d += blockDim.x) {
        const double2 xv = srow[d];
        const uint32_t both = mu & T.md[d];
        const int cd = T.cnt_dn[d];
        double dg = eu + T.ed[d];
        if (UNIFORM_U) {
            dg += T.U0 * (double)__popc(both);
        } else {
            dg += s_U[both & 255u] + s_U[256 + ((both >> 8) & 255u)] + s_U[512 + ((both >> 16) & 255u)];
        }
        double ar = dg * xv.x, ai = dg * xv.y;
        for (int k0 = 0; k0 < cu; k0 += kBatch) {       // up-spin hops: uniform count
            double2 z[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (k0 + j < cu) z[j] = x[s_uprow[k0 + j] + d];
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (k0 + j < cu) {
                    const double tv = s_upval[k0 + j];
                    ar = fma(tv, z[j].x, ar);
                    ai = fma(tv, z[j].y, ai);
                }
        }
        for (int k0 = 0; k0 < cd; k0 += kBatch) {       // down-spin hops: per-lane count
            uint32_t e[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) e[j] = (k0 + j < cd) ? T.ent_dn[(int64_t)(k0 + j) * Ddn + d] : 0u;
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (k0 + j < cd) {
                    double tv = s_negt[(e[j] >> 24) & 127u];
                    tv = (e[j] >> 31) ? -tv : tv;
                    const double2 zz = srow[e[j] & 0xFFFFFFu];
                    ar = fma(tv, zz.x, ar);
                    ai = fma(tv, zz.y, ai);
                }
        }
        double2 out;
        if (MODE == 0) {
            out.x = ar;
            out.y = ai;
        } else {
            out.x = sc * ar;
            out.y = sc * ai;
            if (bp != 0.0) {
                const double2 p = (XP + c * xp_col)[u * Ddn + d];
                out.x = fma(-bp, p.x, out.x);
                out.y = fma(-bp, p.y, out.y);
            }
            dot = fma(sc * xv.x, out.x, dot);
            dot = fma(sc * xv.y, out.y, dot);
        }
        y[u * Ddn + d] = out;
    }
    if (MODE == 1) {
        double s = block_sum(dot, s_red);
        if (tid == 0) part[(int64_t)c * T.Dup + u] = s;
    }
}

// c_alpha / c+_alpha between sectors.  For an up-spin orbital the map is a
// gather of whole rows, for a down-spin orbital a gather inside each row.
__device__ __forceinline__ int64_t rank_of(uint32_t m, const uint64_t* C) {
    int64_t r = 0;
    int k = 1;
    while (m) {
        int p = __ffs(m) - 1;
        r += (int64_t)C[p * kBinomN + k];
        ++k;
        m &= m - 1u;
    }
    return r;
}

__global__ __launch_bounds__(kThreads) void k_apply_c_up(
    const uint32_t* __restrict__ mdst, int64_t Ddn, int site, int dagger,
    const uint64_t* __restrict__ C, const double2* __restrict__ V, int64_t ld_src,
    double2* __restrict__ W, int64_t ld_dst) {
    const int64_t ut = blockIdx.x;
    const int c = blockIdx.y;
    const uint32_t bit = 1u << site;
    const uint32_t mt = mdst[ut];
    // dagger: target has the site occupied, source has it empty (and v.v.)
    const bool ok = dagger ? (mt & bit) != 0u : (mt & bit) == 0u;
    const uint32_t ms = mt ^ bit;
    int64_t us = 0;
    double sign = 0.0;
    if (ok) {
        us = rank_of(ms, C);
        sign = (__popc(ms & (bit - 1u)) & 1) ? -1.0 : 1.0;
    }
    const double2* __restrict__ src = V + c * ld_src + us * Ddn;
    double2* __restrict__ dst = W + c * ld_dst + ut * Ddn;
    for (int64_t d = threadIdx.x; d < Ddn; d += blockDim.x) {
        double2 o = {0.0, 0.0};
        if (ok) {
            double2 z = src[d];
            o.x = sign * z.x;
            o.y = sign * z.y;
        }
        dst[d] = o;
    }
}

__global__ __launch_bounds__(kThreads) void k_apply_c_dn(
    const uint32_t* __restrict__ mdst_dn, int64_t Ddn_src, int64_t Ddn_dst, int site, int dagger,
    int n_up, const uint64_t* __restrict__ C, const double2* __restrict__ V, int64_t ld_src,
    double2* __restrict__ W, int64_t ld_dst) {
    const int64_t u = blockIdx.x;
    const int c = blockIdx.y;
    const uint32_t bit = 1u << site;
    const double2* __restrict__ src = V + c * ld_src + u * Ddn_src;
    double2* __restrict__ dst = W + c * ld_dst + u * Ddn_dst;
    const double upsign = (n_up & 1) ? -1.0 : 1.0;   // all up modes precede down modes
    for (int64_t d = threadIdx.x; d < Ddn_dst; d += blockDim.x) {
        const uint32_t mt = mdst_dn[d];
        const bool ok = dagger ? (mt & bit) != 0u : (mt & bit) == 0u;
        double2 o = {0.0, 0.0};
        if (ok) {
            const uint32_t ms = mt ^ bit;
            const double sign = ((__popc(ms & (bit - 1u)) & 1) ? -1.0 : 1.0) * upsign;
            const double2 z = src[rank_of(ms, C)];
            o.x = sign * z.x;
            o.y = sign * z.y;
        }
        dst[d] = o;
    }
}

template <int MODE>
void launch_hv(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, int ncol,
               const double2* x, int64_t x_col, const double2* xp, int64_t xp_col, double2* y,
               int64_t y_col, const double* s_k, const double* b_k, const double* s_km1,
               int stride, double* part) {
    HvTables T = make_tables(model, sec);
    KGF_REQUIRE(sec->d_up <= 0x7ffffff0 && ncol <= 65535, KGF_EUNSUPPORTED, "H.v: grid too large");
    // algorithmic bytes: read x once, write y once, read xp once if present
    const double vec = 16.0 * (double)sec->dim() * ncol;
    Prof pr(ctx, MODE == 0 ? "hv" : "hv_lanczos", vec * (xp ? 3.0 : 2.0));
    const size_t row_bytes = sizeof(double2) * (size_t)sec->d_dn;
    if (row_bytes <= kRowLdsMax) {
        const int rpx = (int)((sec->d_up + 7) / 8);
        dim3 grid((unsigned)(8 * rpx), (unsigned)ncol);
        // opt in to more than 64 KB of dynamic LDS once per device and kernel
        static bool opted[2][64] = {};
        const int ui = model->U_uniform ? 1 : 0;
        const int dev = ctx->device & 63;
        auto kern = model->U_uniform ? k_hv_lds<MODE, true> : k_hv_lds<MODE, false>;
        if (!opted[ui][dev]) {
            KGF_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowLdsMax));
            opted[ui][dev] = true;
        }
        hipLaunchKernelGGL(kern, grid, dim3(kHvThreads), row_bytes, ctx->stream, T, rpx, x, x_col, xp,
                           xp_col, y, y_col, s_k, b_k, s_km1, stride, part);
        check_launch("k_hv_lds");
        return;
    }
    dim3 grid((unsigned)sec->d_up, (unsigned)ncol);
    if (model->U_uniform)
        hipLaunchKernelGGL((k_hv<MODE, true>), grid, dim3(kThreads), 0, ctx->stream, T, x, x_col, xp,
                           xp_col, y, y_col, s_k, b_k, s_km1, stride, part);
    else
        hipLaunchKernelGGL((k_hv<MODE, false>), grid, dim3(kThreads), 0, ctx->stream, T, x, x_col,
                           xp, xp_col, y, y_col, s_k, b_k, s_km1, stride, part);
    check_launch("k_hv");
}

}  // namespace

void apply_h(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* v, double2* w,
             int nvec, int64_t ld) {
    for (int c0 = 0; c0 < nvec; c0 += 65535) {
        int nc = nvec - c0 < 65535 ? nvec - c0 : 65535;
        launch_hv<0>(ctx, model, sec, nc, v + c0 * ld, ld, nullptr, 0, w + c0 * ld, ld, nullptr,
                     nullptr, nullptr, 0, nullptr);
    }
}

int hv_lanczos_blocks(const kgf_sector* sec) { return (int)sec->d_up; }

void hv_lanczos(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, int ncol,
                const LanczosHvArgs& a) {
    launch_hv<1>(ctx, model, sec, ncol, a.x, a.x_col, a.xp, a.xp_col, a.y, a.y_col, a.s_k, a.b_k,
                 a.s_km1, a.stride, a.part);
}

void apply_c(kgf_ctx* ctx, const kgf_sector* src, const kgf_sector* dst, int orbital, int dagger,
             const double2* v, double2* w, int nvec, int64_t ld_src, int64_t ld_dst) {
    const int site = orbital >> 1, spin = orbital & 1;
    KGF_REQUIRE(dst->d_up <= 0x7fffffff && nvec <= 65535, KGF_EUNSUPPORTED, "c: grid too large");
    dim3 grid((unsigned)dst->d_up, (unsigned)nvec);
    Prof pr(ctx, "apply_c");
    if (spin == 0)
        hipLaunchKernelGGL(k_apply_c_up, grid, dim3(kThreads), 0, ctx->stream,
                           dst->masks_up.as<uint32_t>(), dst->d_dn, site, dagger,
                           ctx->binom.as<uint64_t>(), v, ld_src, w, ld_dst);
    else
        hipLaunchKernelGGL(k_apply_c_dn, grid, dim3(kThreads), 0, ctx->stream,
                           dst->masks_dn.as<uint32_t>(), src->d_dn, dst->d_dn, site, dagger,
                           src->n_up, ctx->binom.as<uint64_t>(), v, ld_src, w, ld_dst);
    check_launch("k_apply_c");
}

}  // namespace kgf
