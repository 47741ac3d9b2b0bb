// Sector basis of a fixed (N_up, N_dn): per spin the L-bit masks with N
// set bits in ascending order (occupation-number basis, Sec. 2; N and S_z
// conservation, Sec. 4).  The position of a mask in that order is its
// combinatorial rank  sum_k C(p_k, k)  over its set bits p_1 < p_2 < ...,
// so the table is built by unranking, in parallel, with integer work only.
#include "kgf_internal.h"

namespace kgf {

int64_t binom_host(int n, int k) {
    if (k < 0 || n < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

void build_binomials(kgf_ctx* ctx) {
    std::vector<uint64_t> c(kBinomN * kBinomN, 0);
    for (int n = 0; n < kBinomN; ++n) {
        c[n * kBinomN] = 1;
        for (int k = 1; k <= n; ++k)
            c[n * kBinomN + k] = c[(n - 1) * kBinomN + k - 1] + (k <= n - 1 ? c[(n - 1) * kBinomN + k] : 0);
    }
    ctx->binom.reserve(sizeof(uint64_t) * c.size());
    KGF_HIP(hipMemcpy(ctx->binom.p, c.data(), sizeof(uint64_t) * c.size(), hipMemcpyHostToDevice));
}

__device__ __forceinline__ uint64_t binom_at(const uint64_t* C, int n, int k) {
    return C[n * kBinomN + k];
}

// rank of a mask among masks of the same popcount (colex = ascending order)
__device__ __forceinline__ int64_t mask_rank(uint32_t m, const uint64_t* C) {
    int64_t r = 0;
    int k = 1;
    while (m) {
        int p = __ffs(m) - 1;
        r += (int64_t)binom_at(C, p, k);
        ++k;
        m &= m - 1u;
    }
    return r;
}

__global__ void k_unrank(uint32_t* __restrict__ masks, int64_t D, int L, int N,
                         const uint64_t* __restrict__ C) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= D) return;
    uint64_t rem = (uint64_t)r;
    uint32_t m = 0;
    int p = L - 1;
    for (int k = N; k >= 1; --k) {
        // largest p with C(p, k) <= rem; C(k-1, k) = 0 bounds the search
        while (binom_at(C, p, k) > rem) --p;
        m |= 1u << p;
        rem -= binom_at(C, p, k);
        --p;
    }
    masks[r] = m;
}

__global__ void k_rank(const uint32_t* __restrict__ masks, int64_t n, int N,
                       const uint64_t* __restrict__ C, int64_t* __restrict__ ranks) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t m = masks[i];
    ranks[i] = (__popc(m) == N) ? mask_rank(m, C) : -1;
}

void build_masks(kgf_ctx* ctx, int L, int n, uint32_t* masks, int64_t D) {
    if (D == 0) return;
    int64_t blocks = (D + kThreads - 1) / kThreads;
    Prof pr(ctx, "sector_unrank");
    hipLaunchKernelGGL(k_unrank, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, masks, D, L,
                       n, ctx->binom.as<uint64_t>());
    check_launch("k_unrank");
}

void rank_masks(kgf_ctx* ctx, const uint32_t* masks, int64_t n, int N, int64_t* ranks) {
    int64_t blocks = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_rank, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, masks, n, N,
                       ctx->binom.as<uint64_t>(), ranks);
    check_launch("k_rank");
}

// ---------------------------------------------------------------------------
// Hopping table of one spin species.  Row r (mask s) lists the masks s'
// with <s| c+_i c_j |s'> != 0 for a bond (i, j) in either direction: exactly
// one of sites i, j is occupied in s, s' = s ^ (1<<i) ^ (1<<j).  Moving one
// fermion past the occupied sites strictly between i and j gives the sign
// (-1)^popcount(s & between(i, j)).  Entries keep the bond index so that the
// amplitude (and, for derivatives, the bond) can be looked up.
// ---------------------------------------------------------------------------
__global__ void k_hop_table(const uint32_t* __restrict__ masks, int64_t D, int nb,
                            const int32_t* __restrict__ bi, const int32_t* __restrict__ bj,
                            const uint64_t* __restrict__ C, int32_t* __restrict__ count,
                            uint32_t* __restrict__ ent, int width) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= D) return;
    uint32_t s = masks[r];
    int c = 0;
    for (int b = 0; b < nb; ++b) {
        int i = bi[b], j = bj[b];
        if ((((s >> i) ^ (s >> j)) & 1u) == 0u) continue;
        uint32_t s2 = s ^ (1u << i) ^ (1u << j);
        int lo = i < j ? i : j, hi = i < j ? j : i;
        uint32_t between = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
        uint32_t sign = (uint32_t)(__popc(s & between) & 1);
        uint32_t col = (uint32_t)mask_rank(s2, C);
        ent[(int64_t)c * D + r] = col | ((uint32_t)b << 24) | (sign << 31);
        ++c;
    }
    count[r] = c;
    for (int k = c; k < width; ++k) ent[(int64_t)k * D + r] = 0u;
}

// per-bond form of the same table: bond[b * D + r] = target | sign << 31, or ~0u
__global__ void k_bond_table(const uint32_t* __restrict__ masks, int64_t D, int nb,
                             const int32_t* __restrict__ bi, const int32_t* __restrict__ bj,
                             const uint64_t* __restrict__ C, uint32_t* __restrict__ out) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= D) return;
    uint32_t s = masks[r];
    for (int b = 0; b < nb; ++b) {
        int i = bi[b], j = bj[b];
        uint32_t v = ~0u;
        if ((((s >> i) ^ (s >> j)) & 1u) != 0u) {
            uint32_t s2 = s ^ (1u << i) ^ (1u << j);
            int lo = i < j ? i : j, hi = i < j ? j : i;
            uint32_t between = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
            uint32_t sign = (uint32_t)(__popc(s & between) & 1);
            v = (uint32_t)mask_rank(s2, C) | (sign << 31);
        }
        out[(int64_t)b * D + r] = v;
    }
}

__global__ void k_onsite(const uint32_t* __restrict__ masks, int64_t D, int L,
                         const double* __restrict__ eu, const double* __restrict__ ed,
                         double* __restrict__ out_up, double* __restrict__ out_dn) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= D) return;
    uint32_t s = masks[r];
    double su = 0.0, sd = 0.0;
    for (int i = 0; i < L; ++i)
        if ((s >> i) & 1u) {
            su += eu[i];
            sd += ed[i];
        }
    out_up[r] = su;
    out_dn[r] = sd;
}

// device copies of a model's parameters: hopping amplitudes and the byte
// tables Utab[q][x] = sum of U_{8q+i} over the set bits i of x
void upload_params(kgf_model* m) {
    m->U_uniform = true;
    for (int i = 1; i < m->L; ++i)
        if (m->U[i] != m->U[0]) m->U_uniform = false;
    m->d_t.reserve(sizeof(double) * (m->nb > 0 ? m->nb : 1));
    if (m->nb) KGF_HIP(hipMemcpy(m->d_t.p, m->t.data(), sizeof(double) * m->nb, hipMemcpyHostToDevice));
    std::vector<double> tab(3 * 256, 0.0);
    for (int q = 0; q < 3; ++q)
        for (int x = 0; x < 256; ++x) {
            double s = 0.0;
            for (int i = 0; i < 8; ++i)
                if (((x >> i) & 1) && 8 * q + i < m->L) s += m->U[8 * q + i];
            tab[q * 256 + x] = s;
        }
    m->d_Utab.reserve(sizeof(double) * tab.size());
    KGF_HIP(hipMemcpy(m->d_Utab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
}

void model_set_params(kgf_model* m, const double* t, const double* eps_up, const double* eps_dn,
                      const double* U) {
    KGF_HIP(hipSetDevice(m->ctx->device));
    KGF_HIP(hipStreamSynchronize(m->ctx->stream));   // issued work keeps the old parameters
    m->t.assign(t, t + m->nb);
    m->eps_up.assign(eps_up, eps_up + m->L);
    m->eps_dn.assign(eps_dn, eps_dn + m->L);
    m->U.assign(U, U + m->L);
    upload_params(m);
    refresh_onsite(m);
    m->version = next_version();
}

// Recompute the on-site energies e_up, e_dn of every hopping table already
// built for the model (after its eps_up / eps_dn changed); the tables'
// targets, bonds and signs depend on the bond topology only.
void refresh_onsite(kgf_model* model) {
    kgf_ctx* ctx = model->ctx;
    if (model->tables.empty()) return;
    DevBuf deu, ded;
    deu.reserve(sizeof(double) * model->L);
    ded.reserve(sizeof(double) * model->L);
    KGF_HIP(hipMemcpyAsync(deu.p, model->eps_up.data(), sizeof(double) * model->L, hipMemcpyHostToDevice,
                           ctx->stream));
    KGF_HIP(hipMemcpyAsync(ded.p, model->eps_dn.data(), sizeof(double) * model->L, hipMemcpyHostToDevice,
                           ctx->stream));
    for (auto& kv : model->tables) {
        HopTable& t = *kv.second;
        if (!t.D) continue;
        const int64_t blocks = (t.D + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_onsite, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, t.masks.as<uint32_t>(),
                           t.D, model->L, deu.as<double>(), ded.as<double>(), t.e_up.as<double>(),
                           t.e_dn.as<double>());
        check_launch("k_onsite");
    }
    sync(ctx);   // the temporaries above are freed on return
}

bool hop_table_ready(const kgf_model* model, int n) { return model->tables.count(n) != 0; }

HopTable& hop_table(kgf_model* model, int n) {
    auto it = model->tables.find(n);
    if (it != model->tables.end()) return *it->second;
    kgf_ctx* ctx = model->ctx;
    std::unique_ptr<HopTable> t(new HopTable());
    t->n = n;
    t->D = binom_host(model->L, n);
    t->width = model->nb;
    KGF_REQUIRE(t->D < (1ll << 24), KGF_EUNSUPPORTED, "hopping table: dimension exceeds 2^24");
    int64_t D = t->D;
    t->masks.reserve(sizeof(uint32_t) * (D ? D : 1));
    t->count.reserve(sizeof(int32_t) * (D ? D : 1));
    t->ent.reserve(sizeof(uint32_t) * (D * t->width ? D * t->width : 1));
    t->e_up.reserve(sizeof(double) * (D ? D : 1));
    t->e_dn.reserve(sizeof(double) * (D ? D : 1));
    t->bond.reserve(sizeof(uint32_t) * (D * model->nb ? D * model->nb : 1));
    if (D) {
        build_masks(ctx, model->L, n, t->masks.as<uint32_t>(), D);
        DevBuf dbi, dbj, deu, ded;
        dbi.reserve(sizeof(int32_t) * (model->nb ? model->nb : 1));
        dbj.reserve(sizeof(int32_t) * (model->nb ? model->nb : 1));
        deu.reserve(sizeof(double) * model->L);
        ded.reserve(sizeof(double) * model->L);
        if (model->nb) {
            KGF_HIP(hipMemcpyAsync(dbi.p, model->bi.data(), sizeof(int32_t) * model->nb,
                                   hipMemcpyHostToDevice, ctx->stream));
            KGF_HIP(hipMemcpyAsync(dbj.p, model->bj.data(), sizeof(int32_t) * model->nb,
                                   hipMemcpyHostToDevice, ctx->stream));
        }
        KGF_HIP(hipMemcpyAsync(deu.p, model->eps_up.data(), sizeof(double) * model->L,
                               hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(ded.p, model->eps_dn.data(), sizeof(double) * model->L,
                               hipMemcpyHostToDevice, ctx->stream));
        int64_t blocks = (D + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_hop_table, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream,
                           t->masks.as<uint32_t>(), D, model->nb, dbi.as<int32_t>(), dbj.as<int32_t>(),
                           ctx->binom.as<uint64_t>(), t->count.as<int32_t>(), t->ent.as<uint32_t>(),
                           t->width);
        check_launch("k_hop_table");
        hipLaunchKernelGGL(k_bond_table, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream,
                           t->masks.as<uint32_t>(), D, model->nb, dbi.as<int32_t>(), dbj.as<int32_t>(),
                           ctx->binom.as<uint64_t>(), t->bond.as<uint32_t>());
        check_launch("k_bond_table");
        hipLaunchKernelGGL(k_onsite, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream,
                           t->masks.as<uint32_t>(), D, model->L, deu.as<double>(), ded.as<double>(),
                           t->e_up.as<double>(), t->e_dn.as<double>());
        check_launch("k_onsite");
        sync(ctx);   // the temporaries above are freed on return
    }
    // Row order of the strip pass: a hop inside either half of the lattice
    // keeps the upper half's particle count, so the rows of one count draw
    // their up-spin sources (all but the few hops across the halves) from the
    // same group, whose strip stays in L2 while it is swept.  Stable counting
    // sort of the ascending masks by that count.
    {
        t->order.reserve(sizeof(int32_t) * (D ? D : 1));
        if (D) {
            const int half = model->L / 2;
            std::vector<int> key((size_t)D);
            std::vector<int64_t> start(model->L + 2, 0);
            uint64_t m = n ? ((uint64_t)1 << n) - 1 : 0;
            for (int64_t r = 0; r < D; ++r) {
                key[(size_t)r] = __builtin_popcountll(m >> half);
                ++start[(size_t)key[(size_t)r] + 1];
                if (m) {   // next mask of the same popcount (ascending)
                    const uint64_t c = m & (~m + 1), rr = m + c;
                    m = (((rr ^ m) >> 2) / c) | rr;
                }
            }
            for (int k = 0; k <= model->L; ++k) start[(size_t)k + 1] += start[(size_t)k];
            std::vector<int32_t> ord((size_t)D);
            for (int64_t r = 0; r < D; ++r) ord[(size_t)start[(size_t)key[(size_t)r]]++] = (int32_t)r;
            KGF_HIP(hipMemcpy(t->order.p, ord.data(), sizeof(int32_t) * (size_t)D, hipMemcpyHostToDevice));
        }
    }
    build_seg_table(model, *t);
    HopTable& ref = *t;
    model->tables[n] = std::move(t);
    return ref;
}

}  // namespace kgf
