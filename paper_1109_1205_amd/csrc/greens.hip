// Green's-function drivers.
//
// Equilibrium (Sec. 3, Eqs. (psit), (psigreen), eta = 0):
//   G^>_{ij}(t) = -i e^{+iE0 t} <c+_i 0| e^{-iHt} |c+_j 0>,
//   G^<_{ij}(t) = +i e^{-iE0 t} <c_j 0| e^{+iHt} |c_i 0>.
// Nonequilibrium four-step procedure (Sec. 4): ground state of H_ini,
// forward states Phi(t_k), backward-propagated Psi_a(t_k) = e^{iHt_k} c_a Phi(t_k)
// for every mesh time, scalar products.  Two schedules of step (iii):
//   plain : each mesh time gets its own backward run (the paper's order);
//   sweep : G^<_{ab}(t_j, t_s) = i <c_b Phi_s| e^{iH(t_j - t_s)} |c_a Phi_j>
//           for j >= s, so one backward sweep from t_max to 0 carries a block
//           of columns X_{a,j}(s) = e^{iH(t_j - t_s)} c_a Phi_j; a column is
//           injected when the sweep reaches t_j and dotted with c_b Phi_s at
//           every later mesh time.  Same number of SIL steps, all columns of
//           the block share every launch.  t_j < t_s follows from
//           G^<_{ab}(t,t')* = -G^<_{ba}(t',t) (same for G^>).
#include <algorithm>
#include <cmath>

#include <cstring>
#include "kgf_internal.h"

namespace kgf {

namespace {

// out[oo + sum_d i_d * os_d] = pref * (cj ? conj : id)(in[io + sum_d i_d * is_d])
struct Map4 {
    int64_t n[4];
    int64_t is[4];
    int64_t os[4];
};

__global__ void k_scatter4(const double2* __restrict__ in, double2* __restrict__ out, Map4 mp,
                           double pre, double pim, int cj) {
    const int64_t total = mp.n[0] * mp.n[1] * mp.n[2] * mp.n[3];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = t;
        int64_t ii = 0, oi = 0;
        for (int d = 3; d >= 0; --d) {
            const int64_t q = r % mp.n[d];
            r /= mp.n[d];
            ii += q * mp.is[d];
            oi += q * mp.os[d];
        }
        double2 z = in[ii];
        if (cj) z.y = -z.y;
        out[oi] = make_double2(pre * z.x - pim * z.y, pre * z.y + pim * z.x);
    }
}

void scatter4(kgf_ctx* ctx, const double2* in, double2* out, const Map4& mp, double pre, double pim, bool cj) {
    const int64_t total = mp.n[0] * mp.n[1] * mp.n[2] * mp.n[3];
    if (total == 0) return;
    int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_scatter4, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, in, out, mp, pre,
                       pim, cj ? 1 : 0);
    check_launch("k_scatter4");
}

// equilibrium: raw[k][i][j] = <X0_i | X_j(t_k)> ->
//   greater: G[k][I][J] = -i e^{+iE0 t_k} raw;  lesser: G[k][J][I] = +i e^{-iE0 t_k} raw
__global__ void k_store_eq(const double2* __restrict__ raw, int nt, int na, int nb_r,
                           const int* __restrict__ gl, const int* __restrict__ gr, int norb,
                           double E0, double tstep, int greater, double2* __restrict__ G) {
    const int64_t total = (int64_t)nt * na * nb_r;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t % nb_r);
        const int i = (int)((t / nb_r) % na);
        const int k = (int)(t / ((int64_t)nb_r * na));
        const double2 z = raw[t];
        const double tk = tstep * k;
        double sn, cs;
        sincos(E0 * tk, &sn, &cs);
        double2 o;
        if (greater) {   // -i (cs + i sn) z
            const double pr = sn, pi = -cs;
            o = make_double2(pr * z.x - pi * z.y, pr * z.y + pi * z.x);
            G[((int64_t)k * norb + gl[i]) * norb + gr[j]] = o;
        } else {         // +i (cs - i sn) z
            const double pr = sn, pi = cs;
            o = make_double2(pr * z.x - pi * z.y, pr * z.y + pi * z.x);
            G[((int64_t)k * norb + gr[j]) * norb + gl[i]] = o;
        }
    }
}

// four-step: raw(s, b, a, j) = <X_b(s) | X_a(j)> with X = c Phi or c+ Phi
// propagated so that the product is <c_b Phi_s| e^{iH(t_j - t_s)} |c_a Phi_j>.
//   lesser : G[j][s][A][B] = +i raw(s, b, a, j)
//   greater: G[j][s][A][B] = -i conj(raw(s, b, a, j))
// half = 1: only j >= s is stored in raw; j < s from G_{AB}(t_j,t_s) = -conj G_{BA}(t_s,t_j)
__global__ void k_store_neq(const double2* __restrict__ raw, int64_t ss, int64_t sb, int64_t sa,
                            int64_t sj, int nt, int na, const int* __restrict__ gidx, int norb,
                            int greater, int half, double2* __restrict__ G) {
    const int64_t total = (int64_t)nt * nt * na * na;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % na);
        const int a = (int)((t / na) % na);
        const int s = (int)((t / ((int64_t)na * na)) % nt);
        const int j = (int)(t / ((int64_t)na * na * nt));
        bool flip = half && j < s;
        double2 z;
        if (!flip)
            z = raw[s * ss + b * sb + a * sa + j * sj];
        else
            z = raw[j * ss + a * sb + b * sa + s * sj];
        double2 g;
        if (greater)
            g = make_double2(-z.y, -z.x);    // -i conj(z)
        else
            g = make_double2(-z.y, z.x);     // +i z
        if (flip) g = make_double2(-g.x, g.y);   // -conj(g)
        G[(((int64_t)j * nt + s) * norb + gidx[a]) * norb + gidx[b]] = g;
    }
}

// sweep bookkeeping: tmp[b][r] for b < nleft, r < ncur, where column
// r = (jhi - j) * nq + q holds orbital q injected at mesh time j
//   -> raw[base + b * sb + q * sa + j * sj]
__global__ void k_place(const double2* __restrict__ tmp, int nleft, int nq, int ncur, int jhi,
                        double2* __restrict__ raw, int64_t base, int64_t sb, int64_t sa, int64_t sj) {
    const int64_t total = (int64_t)nleft * ncur;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t % ncur);
        const int b = (int)(t / ncur);
        const int j = jhi - r / nq, q = r % nq;
        raw[base + b * sb + q * sa + j * sj] = tmp[t];
    }
}

void place(kgf_ctx* ctx, const double2* tmp, int nleft, int nq, int ncur, int jhi, double2* raw, int64_t base,
           int64_t sb, int64_t sa, int64_t sj) {
    const int64_t total = (int64_t)nleft * ncur;
    if (!total) return;
    hipLaunchKernelGGL(k_place, dim3((unsigned)std::min<int64_t>((total + kThreads - 1) / kThreads, 1024)),
                       dim3(kThreads), 0, ctx->stream, tmp, nleft, nq, ncur, jhi, raw, base, sb, sa, sj);
    check_launch("k_place");
}

// mixed component: rawm[(b * ntau + jt) * (na * nt) + a * nt + k] -> Gmix[k][jt][A][B] = i rawm
void store_mixed(kgf_ctx* ctx, const double2* rawm, const std::vector<int>& loc, int nt, int ntau, int norb,
                 double2* Gmix) {
    const int na = (int)loc.size();
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < na; ++b) {
            Map4 m2;
            m2.n[0] = 1; m2.n[1] = ntau; m2.n[2] = 1; m2.n[3] = nt;
            m2.is[0] = 0; m2.is[1] = (int64_t)na * nt; m2.is[2] = 0; m2.is[3] = 1;
            m2.os[0] = 0; m2.os[1] = (int64_t)norb * norb; m2.os[2] = 0; m2.os[3] = (int64_t)ntau * norb * norb;
            const double2* in = rawm + (int64_t)b * ntau * na * nt + (int64_t)a * nt;
            double2* out = Gmix + (int64_t)loc[a] * norb + loc[b];
            scatter4(ctx, in, out, m2, 0.0, 1.0, false);
        }
}

// left mixed component: rawm[(b * ntau + jt) * (na * nt) + a * nt + k] = <P_b(tau_jt) | chi_a(t_k)>
// -> Gmixl[jt][k][A = b][B = a] = -i rawm
void store_mixed_left(kgf_ctx* ctx, const double2* rawm, const std::vector<int>& loc, int nt, int ntau, int norb,
                      double2* Gmixl) {
    const int na = (int)loc.size();
    for (int b = 0; b < na; ++b)
        for (int a = 0; a < na; ++a) {
            Map4 m2;
            m2.n[0] = 1; m2.n[1] = ntau; m2.n[2] = 1; m2.n[3] = nt;
            m2.is[0] = 0; m2.is[1] = (int64_t)na * nt; m2.is[2] = 0; m2.is[3] = 1;
            m2.os[0] = 0; m2.os[1] = (int64_t)nt * norb * norb; m2.os[2] = 0; m2.os[3] = (int64_t)norb * norb;
            const double2* in = rawm + (int64_t)b * ntau * na * nt + (int64_t)a * nt;
            double2* out = Gmixl + (int64_t)loc[b] * norb + loc[a];
            scatter4(ctx, in, out, m2, 0.0, -1.0, false);
        }
}

std::unique_ptr<kgf_sector> make_sector(kgf_ctx* ctx, int L, int nu, int nd) {
    if (nu < 0 || nu > L || nd < 0 || nd > L) return nullptr;
    std::unique_ptr<kgf_sector> s(new kgf_sector());
    s->ctx = ctx;
    s->L = L;
    s->n_up = nu;
    s->n_dn = nd;
    s->d_up = binom_host(L, nu);
    s->d_dn = binom_host(L, nd);
    s->masks_up.reserve(sizeof(uint32_t) * s->d_up);
    s->masks_dn.reserve(sizeof(uint32_t) * s->d_dn);
    build_masks(ctx, L, nu, s->masks_up.as<uint32_t>(), s->d_up);
    build_masks(ctx, L, nd, s->masks_dn.as<uint32_t>(), s->d_dn);
    return s;
}

std::unique_ptr<kgf_sector> shifted(kgf_ctx* ctx, const kgf_sector* sec, int spin, int delta) {
    return make_sector(ctx, sec->L, sec->n_up + (spin == 0 ? delta : 0), sec->n_dn + (spin == 1 ? delta : 0));
}

void upload_ints(kgf_ctx* ctx, DevBuf& buf, const std::vector<int>& v) {
    buf.reserve(sizeof(int) * (v.empty() ? 1 : v.size()));
    if (!v.empty()) KGF_HIP(hipMemcpy(buf.p, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
}

void release(kgf_ctx* ctx, const char* name) {
    auto it = ctx->ws.find(name);
    if (it != ctx->ws.end()) {
        sync(ctx);
        ctx->ws.erase(it);
    }
}

}  // namespace

void greens_eq(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0, double E0,
               const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o, int batch,
               double2* Gg_host, double2* Gl_host) {
    TraceRange range_("kgf equilibrium G");
    const size_t gsz = sizeof(double2) * (size_t)nt * norb * norb;
    double2* Gdev = static_cast<double2*>(workspace(ctx, "geq_G", 2 * gsz));
    KGF_HIP(hipMemsetAsync(Gdev, 0, 2 * gsz, ctx->stream));
    const double tstep = spg * o.dt;
    for (int spin = 0; spin < 2; ++spin) {
        std::vector<int> loc;
        for (int a = 0; a < norb; ++a)
            if ((orbs[a] & 1) == spin) loc.push_back(a);
        const int na = (int)loc.size();
        if (!na) continue;
        for (int greater = 1; greater >= 0; --greater) {
            auto tgt = shifted(ctx, sec, spin, greater ? +1 : -1);
            if (!tgt || tgt->dim() == 0) continue;
            const int64_t Dt = tgt->dim();
            double2* X0 = static_cast<double2*>(workspace(ctx, "geq_X0", sizeof(double2) * na * Dt));
            double2* Xt = static_cast<double2*>(workspace(ctx, "geq_Xt", sizeof(double2) * na * Dt));
            double2* raw = static_cast<double2*>(workspace(ctx, "geq_raw", sizeof(double2) * (size_t)nt * na * na));
            for (int q = 0; q < na; ++q)
                apply_c(ctx, sec, tgt.get(), orbs[loc[q]], greater, psi0, X0 + q * Dt, 1, sec->dim(), Dt);
            KGF_HIP(hipMemcpyAsync(Xt, X0, sizeof(double2) * na * Dt, hipMemcpyDeviceToDevice, ctx->stream));
            SilOpts so = o;
            so.direction = greater ? -1 : +1;
            const int B = (batch <= 0 || batch > na) ? na : batch;
            for (int c0 = 0; c0 < na; c0 += B) {
                const int nc = std::min(B, na - c0);
                for (int k = 0; k < nt; ++k) {
                    if (k > 0) sil_propagate(ctx, model, tgt.get(), Xt + c0 * Dt, nc, Dt, spg, so);
                    // raw[k][i][c0 + j] = <X0_i | Xt_j>
                    block_dots(ctx, X0, Dt, na, Xt + c0 * Dt, Dt, nc, Dt, raw + (size_t)k * na * na + c0, na);
                    progress(ctx, greater ? "eq_greater" : "eq_lesser", (int64_t)c0 * nt + (int64_t)(k + 1) * nc,
                             (int64_t)na * nt);
                }
            }
            DevBuf gl;
            upload_ints(ctx, gl, loc);
            int64_t total = (int64_t)nt * na * na;
            int64_t blocks = std::min<int64_t>((total + kThreads - 1) / kThreads, 4096);
            hipLaunchKernelGGL(k_store_eq, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, raw, nt, na, na,
                               gl.as<int>(), gl.as<int>(), norb, E0, tstep, greater,
                               Gdev + (greater ? 0 : (size_t)nt * norb * norb));
            check_launch("k_store_eq");
            sync(ctx);
        }
    }
    if (Gg_host) KGF_HIP(hipMemcpyAsync(Gg_host, Gdev, gsz, hipMemcpyDeviceToHost, ctx->stream));
    if (Gl_host)
        KGF_HIP(hipMemcpyAsync(Gl_host, Gdev + (size_t)nt * norb * norb, gsz, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
}

// The forward mesh Phi(t_k) = exp(-iH t_k)|0>, k < nt.  Stored whole when it
// fits; otherwise only every K-th state is kept (checkpoints) and the states
// in between are recomputed, one segment of K - 1 states at a time, by the
// same forward steps (so every Phi(t_k) is bitwise the stored-mesh value).
// Accesses that walk k monotonically recompute each segment once.
struct PhiMesh {
    kgf_ctx* ctx = nullptr;
    kgf_model* H = nullptr;
    const kgf_sector* sec = nullptr;
    SilOpts fo;
    int spg = 1, nt = 0, K = 1;
    int64_t D = 0;
    double2* ck = nullptr;    // K == 1: all nt states; else ceil(nt / K) checkpoints
    double2* seg = nullptr;   // K - 1 states after the current checkpoint
    int seg_id = -1;

    const double2* at(int k) {
        if (K == 1) return ck + (size_t)k * D;
        const int c = k / K, i = k % K;
        if (i == 0) return ck + (size_t)c * D;
        if (seg_id != c) {
            for (int r = 1; r < K && c * K + r < nt; ++r) {
                double2* dst = seg + (size_t)(r - 1) * D;
                const double2* src = r == 1 ? ck + (size_t)c * D : dst - D;
                KGF_HIP(hipMemcpyAsync(dst, src, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
                sil_propagate(ctx, H, sec, dst, 1, D, spg, fo);
            }
            seg_id = c;
        }
        return seg + (size_t)(i - 1) * D;
    }
};

struct NeqArgs {
    kgf_model* H_ini;
    kgf_model* H;
    const kgf_sector* sec;
    const int32_t* orbs;
    int norb, nt, spg;
    SilOpts o;
    int schedule, batch;
    int ntau, tspg;
    double dtau;
};

// Step (iii)+(iv) of one spin group and one operator (c or c+) in the sweep
// schedule, advanced one mesh interval at a time.  Columns are injected in
// chunks of source times [jlo, jhi] (chunk width from `batch` or free
// memory); interval() takes the block at t_s: injects c_a Phi(t_s) when
// s is in the chunk, dots every column with c_b Phi(t_s) and moves the
// block to t_{s-1} (one SIL step per grid step).  finish() stores G.
struct SweepBranch {
    kgf_ctx* ctx = nullptr;
    const NeqArgs* A = nullptr;
    std::vector<int> loc;
    int dagger = 0, na = 0, nt = 0;
    std::unique_ptr<kgf_sector> tgt;
    int64_t D = 0, Dt = 0;
    SilOpts so;
    DevBuf gidx;
    double2 *raw = nullptr, *rawm = nullptr, *S = nullptr, *Lb = nullptr, *tmp = nullptr;
    // mixed component: states on the tau mesh (or null) -- e^{-(H_ini-E0) tau} c_b |0> for the c
    // sweep (G^|(t, tau)), e^{-(H_ini-E0) tau} c+_b |0> for the c+ sweep (G^|(tau, t))
    const double2* hole = nullptr;
    int jchunk = 1, jhi = -1, jlo = 0, s = 0, ncur = 0;
    bool in_chunk = false;
    int64_t ss = 0, sb = 0, sa = 0, sj = 1;

    // false when the operator's target sector is empty (nothing to do)
    bool begin(kgf_ctx* c, const NeqArgs& args, const std::vector<int>& orbs_loc, int spin, int dag,
               const double2* hole_states) {
        ctx = c;
        A = &args;
        loc = orbs_loc;
        dagger = dag;
        const kgf_sector* sec = A->sec;
        tgt = shifted(ctx, sec, spin, dagger ? +1 : -1);
        if (!tgt || tgt->dim() == 0) return false;
        D = sec->dim();
        Dt = tgt->dim();
        na = (int)loc.size();
        nt = A->nt;
        so = A->o;
        so.direction = +1;   // e^{+iH dt}
        upload_ints(ctx, gidx, loc);
        raw = static_cast<double2*>(workspace(ctx, "neq_raw", sizeof(double2) * (size_t)nt * nt * na * na));
        KGF_HIP(hipMemsetAsync(raw, 0, sizeof(double2) * (size_t)nt * nt * na * na, ctx->stream));
        hole = hole_states;
        if (hole)
            rawm = static_cast<double2*>(workspace(ctx, "neq_rawm", sizeof(double2) * (size_t)na * A->ntau * na * nt));
        const size_t per_col = sizeof(double2) * (size_t)(A->o.m + 1) * Dt;
        int Bcols = A->batch;
        if (Bcols <= 0) {
            size_t free_b = 0, total_b = 0;
            KGF_HIP(hipMemGetInfo(&free_b, &total_b));
            const size_t budget = (size_t)(0.80 * (double)free_b);
            Bcols = (int)std::max<size_t>(1, budget / per_col);
        }
        if (A->batch <= 0 && ctx->hv_tune) {
            // widths as multiples of the spin group: the block of one source time
            const int w = tuned_sweep_width(ctx, A->H, tgt.get(), std::min(Bcols, nt * na), so);
            Bcols = std::max(na, (w / na) * na);
        }
        jchunk = std::min(std::max(1, Bcols / na), nt);
        const int maxcols = jchunk * na;
        release(ctx, "sil_X");
        sil_reserve(ctx, tgt.get(), maxcols, A->o.m, A->o.reorth);
        ensure_device_fits(sizeof(double2) * (size_t)maxcols * Dt, "four-step sweep block");
        S = static_cast<double2*>(workspace(ctx, "neq_cols", sizeof(double2) * (size_t)maxcols * Dt));
        Lb = static_cast<double2*>(workspace(ctx, "neq_left", sizeof(double2) * (size_t)na * Dt));
        tmp = static_cast<double2*>(workspace(ctx, "neq_tmp", sizeof(double2) * (size_t)na * maxcols));
        // raw layout [s][b][a][j]
        ss = (int64_t)na * na * nt;
        sb = (int64_t)na * nt;
        sa = nt;
        sj = 1;
        jhi = nt - 1;
        in_chunk = false;
        return true;
    }

    bool finished() const { return jhi < 0; }
    // columns the next interval works on (after its injection), its mesh
    // index s, and the full width of the chunk it belongs to
    int next_width() const {
        if (finished()) return 0;
        if (!in_chunk) return na;
        return ncur + (s >= jlo ? na : 0);
    }
    int next_s() const { return finished() ? -1 : (in_chunk ? s : jhi); }
    int chunk_width() const {
        if (finished()) return 0;
        return (jhi - std::max(0, jhi - jchunk + 1) + 1) * na;
    }

    // one mesh interval; returns the SIL column-steps it ran
    int64_t interval(PhiMesh& Phi) {
        TraceRange range_("kgf sweep interval");
        const kgf_sector* sec = A->sec;
        if (!in_chunk) {
            jlo = std::max(0, jhi - jchunk + 1);
            ncur = 0;   // column r = (jhi - j) * na + q holds X_{q, j}
            s = jhi;
            in_chunk = true;
        }
        if (s >= jlo) {
            for (int q = 0; q < na; ++q)
                apply_c(ctx, sec, tgt.get(), A->orbs[loc[q]], dagger, Phi.at(s), S + (size_t)(ncur + q) * Dt, 1, D,
                        Dt);
            ncur += na;
        }
        for (int q = 0; q < na; ++q)
            apply_c(ctx, sec, tgt.get(), A->orbs[loc[q]], dagger, Phi.at(s), Lb + (size_t)q * Dt, 1, D, Dt);
        // tmp[b][r] = <c_b Phi_s | X_r>
        block_dots(ctx, Lb, Dt, na, S, Dt, ncur, Dt, tmp, ncur);
        place(ctx, tmp, na, na, ncur, jhi, raw, s * ss, sb, sa, sj);
        int64_t steps = 0;
        if (s > 0) {
            sil_propagate(ctx, A->H, tgt.get(), S, ncur, Dt, A->spg, so);
            steps = (int64_t)ncur * A->spg;
        }
        progress(ctx, dagger ? "sweep_greater" : "sweep_lesser", jhi - s + 1, jhi + 1);
        if (--s < 0) {   // chunk done: the columns hold Psi_a(t_j), j in [jlo, jhi]
            if (hole) {
                double2* tmpm =
                    static_cast<double2*>(workspace(ctx, "neq_tmpm", sizeof(double2) * (size_t)na * A->ntau * ncur));
                block_dots(ctx, hole, Dt, na * A->ntau, S, Dt, ncur, Dt, tmpm, ncur);
                // rawm layout [(b, jt)][a][k]: (b, jt) is the "left" index of place()
                place(ctx, tmpm, na * A->ntau, na, ncur, jhi, rawm, 0, (int64_t)na * nt, nt, 1);
            }
            jhi -= jchunk;
            in_chunk = false;
        }
        return steps;
    }

    void finish(double2* Gdev, double2* Gmix_dev) {
        const int64_t total = (int64_t)nt * nt * na * na;
        hipLaunchKernelGGL(k_store_neq, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(kThreads),
                           0, ctx->stream, raw, ss, sb, sa, sj, nt, na, gidx.as<int>(), A->norb, dagger, 1, Gdev);
        check_launch("k_store_neq");
        if (hole && Gmix_dev) {
            if (dagger) store_mixed_left(ctx, rawm, loc, nt, A->ntau, A->norb, Gmix_dev);
            else store_mixed(ctx, rawm, loc, nt, A->ntau, A->norb, Gmix_dev);
        }
    }
};

// step (iii)+(iv) for one spin group and one operator (c or c+); also a
// mixed component when `Gmix_dev` is given: G^|(t, tau) from the c sweep
// with the hole states, G^|(tau, t) from the c+ sweep with the particle
// states (`tau_states`, on the tau mesh).
static void neq_branch(kgf_ctx* ctx, const NeqArgs& A, const std::vector<int>& loc, int spin, int dagger,
                       PhiMesh& Phi, double2* Gdev, const double2* tau_states, double2* Gmix_dev) {
    const bool want_mixed = (Gmix_dev != nullptr && A.ntau > 0 && tau_states);
    const double2* hole_states = tau_states;
    if (A.schedule == 1) {
        SweepBranch br;
        if (!br.begin(ctx, A, loc, spin, dagger, want_mixed ? hole_states : nullptr)) return;
        while (!br.finished()) br.interval(Phi);
        br.finish(Gdev, want_mixed ? Gmix_dev : nullptr);
        sync(ctx);
        return;
    }
    const kgf_sector* sec = A.sec;
    auto tgt = shifted(ctx, sec, spin, dagger ? +1 : -1);
    if (!tgt || tgt->dim() == 0) return;
    const int64_t D = sec->dim();
    const int64_t Dt = tgt->dim();
    const int na = (int)loc.size();
    const int nt = A.nt;
    SilOpts so = A.o;
    so.direction = +1;   // e^{+iH dt}
    DevBuf gidx;
    upload_ints(ctx, gidx, loc);
    double2* raw = static_cast<double2*>(workspace(ctx, "neq_raw", sizeof(double2) * (size_t)nt * nt * na * na));
    KGF_HIP(hipMemsetAsync(raw, 0, sizeof(double2) * (size_t)nt * nt * na * na, ctx->stream));
    double2* rawm = nullptr;
    if (want_mixed)
        rawm = static_cast<double2*>(workspace(ctx, "neq_rawm", sizeof(double2) * (size_t)na * A.ntau * na * nt));

    if (A.schedule == 0) {
        // literal: Psi_a(t_k) for every mesh time, then all scalar products
        const size_t bytes = sizeof(double2) * (size_t)na * nt * Dt;
        ensure_device_fits(bytes, "four-step (plain) state mesh");
        double2* Psi = static_cast<double2*>(workspace(ctx, "neq_psi", bytes));
        for (int q = 0; q < na; ++q)
            for (int k = 0; k < nt; ++k) {
                double2* x = Psi + ((size_t)q * nt + k) * Dt;
                apply_c(ctx, sec, tgt.get(), A.orbs[loc[q]], dagger, Phi.at(k), x, 1, D, Dt);
                if (k > 0) sil_propagate(ctx, A.H, tgt.get(), x, 1, Dt, k * A.spg, so);
                progress(ctx, dagger ? "backward_greater" : "backward_lesser", (int64_t)q * nt + k + 1,
                         (int64_t)na * nt);
            }
        // raw layout [b][s][a][j] = <Psi_b(s) | Psi_a(j)>
        block_dots(ctx, Psi, Dt, na * nt, Psi, Dt, na * nt, Dt, raw, (int64_t)na * nt);
        const int64_t ss = na * nt, sb = (int64_t)nt * na * nt, sa = nt, sj = 1;
        int64_t total = (int64_t)nt * nt * na * na;
        hipLaunchKernelGGL(k_store_neq, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(kThreads), 0,
                           ctx->stream, raw, ss, sb, sa, sj, nt, na, gidx.as<int>(), A.norb, dagger, 0, Gdev);
        check_launch("k_store_neq");
        if (want_mixed) {
            // rawm[(b, jt)][(a, k)] = <state_b(tau_jt) | Psi_a(t_k)> (chi_a(t_k) for c+)
            block_dots(ctx, hole_states, Dt, na * A.ntau, Psi, Dt, na * nt, Dt, rawm, (int64_t)na * nt);
            if (dagger) store_mixed_left(ctx, rawm, loc, nt, A.ntau, A.norb, Gmix_dev);
            else store_mixed(ctx, rawm, loc, nt, A.ntau, A.norb, Gmix_dev);
        }
        sync(ctx);
        release(ctx, "neq_psi");
    }
}

// Grid points between stored forward states: 1 (store all) when the mesh
// takes at most 35% of free device memory, else the smallest K whose
// checkpoints plus one segment take at most 30%; kgf_set_option can fix K.
static int phi_checkpoint_interval(kgf_ctx* ctx, int nt, int64_t D) {
    if (ctx->phi_every > 0) return std::min(ctx->phi_every, std::max(nt, 1));
    size_t free_b = 0, total_b = 0;
    KGF_HIP(hipMemGetInfo(&free_b, &total_b));
    const double vb = 16.0 * (double)D;
    if (vb * nt <= 0.35 * (double)free_b) return 1;
    for (int K = 2; K <= nt; ++K) {
        const int nck = (nt + K - 1) / K;
        if (vb * (nck + K - 1) <= 0.30 * (double)free_b) return K;
    }
    return std::max(nt, 1);
}

// Steps (i) and (ii): ground state of H_ini (returned, also copied to
// psi0_out when given) and the forward mesh Phi(t_k), whole or as checkpoints.
static double2* neq_forward(kgf_ctx* ctx, const NeqArgs& A, const double2* v0, const kgf_gs_opts* gso,
                            double* E0_out, double2* psi0_out, PhiMesh& Phi) {
    TraceRange range_("kgf forward mesh");
    const kgf_sector* sec = A.sec;
    const int64_t D = sec->dim();
    const int nt = A.nt;
    // (i) ground state of H_ini
    double2* psi0 = static_cast<double2*>(workspace(ctx, "neq_psi0", sizeof(double2) * D));
    GsResult gs = ground_state(ctx, A.H_ini, sec, v0, psi0, gso->tol, gso->max_iter, gso->check_every, gso->reorth);
    release(ctx, "gs_V");
    release(ctx, "gs_partbig");
    KGF_REQUIRE(gs.converged, KGF_ENOCONV, "four-step: ground state of H_ini did not converge");
    require_unique_ground_state(ctx, A.H_ini, sec, psi0, gso, "four-step");
    *E0_out = gs.E0;
    if (psi0_out)
        KGF_HIP(hipMemcpyAsync(psi0_out, psi0, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
    // (ii) forward states on the mesh (whole, or checkpoints every K)
    Phi.ctx = ctx;
    Phi.H = A.H;
    Phi.sec = sec;
    Phi.fo = A.o;
    Phi.fo.direction = -1;
    Phi.spg = A.spg;
    Phi.nt = nt;
    Phi.D = D;
    Phi.K = phi_checkpoint_interval(ctx, nt, D);
    const int nck = (nt + Phi.K - 1) / Phi.K;
    const size_t vb = sizeof(double2) * (size_t)D;
    ensure_device_fits(vb * (size_t)(nck + (Phi.K > 1 ? Phi.K - 1 : 0)), "four-step forward mesh");
    Phi.ck = static_cast<double2*>(workspace(ctx, "neq_phi", vb * (size_t)nck));
    if (Phi.K > 1) Phi.seg = static_cast<double2*>(workspace(ctx, "neq_phiseg", vb * (size_t)(Phi.K - 1)));
    KGF_HIP(hipMemcpyAsync(Phi.ck, psi0, vb, hipMemcpyDeviceToDevice, ctx->stream));
    {
        // running state: the mesh itself (K == 1) or the first segment slot
        double2* run = Phi.K == 1 ? Phi.ck : Phi.seg;
        if (Phi.K > 1) KGF_HIP(hipMemcpyAsync(run, psi0, vb, hipMemcpyDeviceToDevice, ctx->stream));
        for (int k = 1; k < nt; ++k) {
            if (Phi.K == 1) {
                KGF_HIP(hipMemcpyAsync(Phi.ck + (size_t)k * D, Phi.ck + (size_t)(k - 1) * D, vb,
                                       hipMemcpyDeviceToDevice, ctx->stream));
                sil_propagate(ctx, A.H, sec, Phi.ck + (size_t)k * D, 1, D, A.spg, Phi.fo);
            } else {
                sil_propagate(ctx, A.H, sec, run, 1, D, A.spg, Phi.fo);
                if (k % Phi.K == 0)
                    KGF_HIP(hipMemcpyAsync(Phi.ck + (size_t)(k / Phi.K) * D, run, vb, hipMemcpyDeviceToDevice,
                                           ctx->stream));
            }
            progress(ctx, "forward", k, nt - 1);
        }
    }
    return psi0;
}

void greens_neq(kgf_ctx* ctx, const NeqArgs& A, const double2* v0, const kgf_gs_opts* gso, double* E0_out,
                double2* psi0_out, double2* Gl_host, double2* Gg_host, double2* GM_host, double2* Gmix_host,
                double2* Gmixl_host) {
    TraceRange range_("kgf four-step");
    const kgf_sector* sec = A.sec;
    const int64_t D = sec->dim();
    const int nt = A.nt, norb = A.norb;
    PhiMesh Phi;
    const double2* psi0 = neq_forward(ctx, A, v0, gso, E0_out, psi0_out, Phi);
    const double E0 = *E0_out;
    const size_t gsz = sizeof(double2) * (size_t)nt * nt * norb * norb;
    double2* Gl = static_cast<double2*>(workspace(ctx, "neq_Gl", gsz));
    double2* Gg = static_cast<double2*>(workspace(ctx, "neq_Gg", gsz));
    KGF_HIP(hipMemsetAsync(Gl, 0, gsz, ctx->stream));
    KGF_HIP(hipMemsetAsync(Gg, 0, gsz, ctx->stream));
    const bool matsubara = A.ntau > 0 && (GM_host || Gmix_host || Gmixl_host);
    const size_t gmsz = sizeof(double2) * 2 * (size_t)std::max(A.ntau, 1) * norb * norb;
    const size_t gxsz = sizeof(double2) * (size_t)nt * std::max(A.ntau, 1) * norb * norb;
    double2* GM = static_cast<double2*>(workspace(ctx, "neq_GM", gmsz));
    double2* Gx = static_cast<double2*>(workspace(ctx, "neq_Gx", gxsz));
    double2* Gxl = static_cast<double2*>(workspace(ctx, "neq_Gxl", gxsz));
    KGF_HIP(hipMemsetAsync(GM, 0, gmsz, ctx->stream));
    KGF_HIP(hipMemsetAsync(Gx, 0, gxsz, ctx->stream));
    KGF_HIP(hipMemsetAsync(Gxl, 0, gxsz, ctx->stream));
    SilOpts io = A.o;
    io.direction = 0;
    io.shift = E0;
    io.dt = A.dtau;
    for (int spin = 0; spin < 2; ++spin) {
        std::vector<int> loc;
        for (int a = 0; a < norb; ++a)
            if ((A.orbs[a] & 1) == spin) loc.push_back(a);
        const int na = (int)loc.size();
        if (!na) continue;
        // Matsubara branch with H_ini: particle (c+) and hole (c) states on the tau mesh
        double2* hole = nullptr;
        double2* particle = nullptr;
        if (matsubara) {
            for (int part = 0; part < 2; ++part) {   // part 0: particle (c+), 1: hole (c)
                auto ts = shifted(ctx, sec, spin, part == 0 ? +1 : -1);
                if (!ts || ts->dim() == 0) continue;
                const int64_t Dt = ts->dim();
                const size_t bytes = sizeof(double2) * (size_t)na * A.ntau * Dt;
                ensure_device_fits(bytes, "Matsubara mesh");
                double2* P = static_cast<double2*>(workspace(ctx, part == 0 ? "neq_mats_p" : "neq_mats_h", bytes));
                double2* X0 = static_cast<double2*>(workspace(ctx, "neq_mats_x0", sizeof(double2) * na * Dt));
                for (int q = 0; q < na; ++q) {
                    apply_c(ctx, sec, ts.get(), A.orbs[loc[q]], part == 0 ? 1 : 0, psi0, X0 + q * Dt, 1, D, Dt);
                    KGF_HIP(hipMemcpyAsync(P + (size_t)q * A.ntau * Dt, X0 + q * Dt, sizeof(double2) * Dt,
                                           hipMemcpyDeviceToDevice, ctx->stream));
                    for (int j = 1; j < A.ntau; ++j) {
                        double2* x = P + ((size_t)q * A.ntau + j) * Dt;
                        KGF_HIP(hipMemcpyAsync(x, x - Dt, sizeof(double2) * Dt, hipMemcpyDeviceToDevice, ctx->stream));
                        sil_propagate(ctx, A.H_ini, ts.get(), x, 1, Dt, A.tspg, io);
                    }
                }
                // rawp[l][(b, j)] = <X0_l | P_b(tau_j)>
                double2* rawp = static_cast<double2*>(workspace(ctx, "neq_rawp", sizeof(double2) * (size_t)na * na * A.ntau));
                block_dots(ctx, X0, Dt, na, P, Dt, na * A.ntau, Dt, rawp, (int64_t)na * A.ntau);
                for (int l = 0; l < na; ++l)
                    for (int b = 0; b < na; ++b) {
                        Map4 m2;
                        m2.n[0] = 1; m2.n[1] = 1; m2.n[2] = 1; m2.n[3] = A.ntau;
                        m2.is[0] = m2.is[1] = m2.is[2] = 0; m2.is[3] = 1;
                        m2.os[0] = m2.os[1] = m2.os[2] = 0; m2.os[3] = (int64_t)norb * norb;
                        const double2* in = rawp + ((size_t)l * na + b) * A.ntau;
                        if (part == 0) {   // G^M(+tau)[j][A=l][B=b] = -<c+_A 0|P_B>
                            double2* out = GM + (int64_t)loc[l] * norb + loc[b];
                            scatter4(ctx, in, out, m2, -1.0, 0.0, false);
                        } else {           // G^M(-tau)[j][A=b][B=l] = <c_B 0| H_A>
                            double2* out = GM + (size_t)A.ntau * norb * norb + (int64_t)loc[b] * norb + loc[l];
                            scatter4(ctx, in, out, m2, 1.0, 0.0, false);
                        }
                    }
                sync(ctx);
                (part == 0 ? particle : hole) = P;
            }
        }
        for (int dagger = 0; dagger < 2; ++dagger) {
            // G^|(t, tau) from the c sweep, G^|(tau, t) from the c+ sweep
            double2* mix = nullptr;
            if (matsubara) mix = dagger ? (Gmixl_host ? Gxl : nullptr) : (Gmix_host ? Gx : nullptr);
            neq_branch(ctx, A, loc, spin, dagger, Phi, dagger ? Gg : Gl, dagger ? particle : hole, mix);
        }
        release(ctx, "neq_mats_p");
        release(ctx, "neq_mats_h");
    }
    if (Gl_host) KGF_HIP(hipMemcpyAsync(Gl_host, Gl, gsz, hipMemcpyDeviceToHost, ctx->stream));
    if (Gg_host) KGF_HIP(hipMemcpyAsync(Gg_host, Gg, gsz, hipMemcpyDeviceToHost, ctx->stream));
    if (matsubara && GM_host)
        KGF_HIP(hipMemcpyAsync(GM_host, GM, sizeof(double2) * 2 * (size_t)A.ntau * norb * norb,
                               hipMemcpyDeviceToHost, ctx->stream));
    if (matsubara && Gmix_host)
        KGF_HIP(hipMemcpyAsync(Gmix_host, Gx, sizeof(double2) * (size_t)nt * A.ntau * norb * norb,
                               hipMemcpyDeviceToHost, ctx->stream));
    if (matsubara && Gmixl_host)
        KGF_HIP(hipMemcpyAsync(Gmixl_host, Gxl, sizeof(double2) * (size_t)nt * A.ntau * norb * norb,
                               hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    release(ctx, "neq_Gxl");
    release(ctx, "neq_phi");
    release(ctx, "neq_phiseg");
    release(ctx, "neq_cols");
    release(ctx, "sil_X");
}

// Four-step G^<, G^> (sweep schedule) for several instances at once.
// Instances with equal sectors and bond topologies form a group; a group's
// forward meshes and backward sweeps run as one multi-column batch in which
// column c carries the Hamiltonian of member c mod n (ModelSet), so every
// launch serves all members.  Ground states are found per instance.
// Gl_host / Gg_host: [ninst][nt][nt][norb][norb]; E0_host: [ninst].
// Lockstep form of the same computation: every group's ground states first,
// then the forward meshes and the backward sweeps of all groups advance
// together, each SIL step one grouped launch per kernel over the columns of
// every group (sectors of different size, a Hamiltonian per column).  The
// sweeps share one chunk of source times sized for all groups.  Per group
// the kernels, element owners and reduction orders are those of the
// group-by-group path, so the results are the same.
struct LockGroup {
    std::vector<int> mem;                  // instance indices
    const kgf_sector* sec = nullptr;
    std::unique_ptr<ModelSet> set;
    double2* Phi = nullptr;                // [nt][n][D]
    std::unique_ptr<kgf_sector> tgt;       // target sector of the current branch
    double2 *raw = nullptr, *S = nullptr, *Lb = nullptr, *tmp = nullptr;
    std::vector<double2> Gl, Gg;           // host [n][nt][nt][norb][norb]
};

static bool lockstep_possible(kgf_ctx* ctx, int ninst, kgf_model* const* Hf, const kgf_sector* const* secs,
                              const SilOpts& o) {
    if (o.reorth != 0) return false;
    std::vector<GroupSpec> probe;
    std::vector<std::unique_ptr<kgf_sector>> keep;
    for (int i = 0; i < ninst; ++i) {
        probe.push_back(GroupSpec{HModel(Hf[i]), secs[i], 0, 1});
        for (int spin = 0; spin < 2; ++spin)
            for (int d = -1; d <= 1; d += 2) {
                auto t = shifted(ctx, secs[i], spin, d);
                if (t && t->dim() > 0) {
                    probe.push_back(GroupSpec{HModel(Hf[i]), t.get(), 0, 1});
                    keep.push_back(std::move(t));
                }
            }
    }
    return hv_groups_supported(ctx, probe);
}

static void greens_neq_multi_lockstep(kgf_ctx* ctx, int ninst, kgf_model* const* Hi, kgf_model* const* Hf,
                                      const kgf_sector* const* secs, const double2* const* v0,
                                      const kgf_gs_opts* gso, const int32_t* orbs, int norb, int nt, int spg,
                                      const SilOpts& o, int batch, double2* Gl_host, double2* Gg_host,
                                      double* E0_host) {
    std::vector<int> done(ninst, 0);
    std::vector<LockGroup> G;
    for (int i0 = 0; i0 < ninst; ++i0) {
        if (done[i0]) continue;
        LockGroup g;
        for (int i = i0; i < ninst; ++i)
            if (!done[i] && secs[i]->L == secs[i0]->L && secs[i]->n_up == secs[i0]->n_up &&
                secs[i]->n_dn == secs[i0]->n_dn && same_topology(Hf[i], Hf[i0])) {
                g.mem.push_back(i);
                done[i] = 1;
            }
        g.sec = secs[i0];
        g.set.reset(new ModelSet());
        for (int i : g.mem) g.set->models.push_back(Hf[i]);
        model_set_init(ctx, *g.set);
        G.push_back(std::move(g));
    }
    const size_t gsz = (size_t)nt * nt * norb * norb;
    // (i) ground states, one instance at a time, into the first mesh slot
    size_t phi_bytes = 0;
    for (auto& g : G) phi_bytes += sizeof(double2) * (size_t)nt * g.mem.size() * g.sec->dim();
    ensure_device_fits(phi_bytes, "batched four-step forward meshes");
    for (size_t gi = 0; gi < G.size(); ++gi) {
        LockGroup& g = G[gi];
        const int n = (int)g.mem.size();
        const int64_t D = g.sec->dim();
        g.Phi = static_cast<double2*>(workspace(ctx, "lneq_phi" + std::to_string(gi),
                                                sizeof(double2) * (size_t)nt * n * D));
        for (int k = 0; k < n; ++k) {
            GsResult gs = ground_state(ctx, Hi[g.mem[k]], g.sec, v0[g.mem[k]], g.Phi + (size_t)k * D, gso->tol,
                                       gso->max_iter, gso->check_every, gso->reorth);
            KGF_REQUIRE(gs.converged, KGF_ENOCONV, "batched four-step: a ground state of H_ini did not converge");
            require_unique_ground_state(ctx, Hi[g.mem[k]], g.sec, g.Phi + (size_t)k * D, gso, "batched four-step");
            E0_host[g.mem[k]] = gs.E0;
        }
        progress(ctx, "ground_states", gi + 1, G.size());
        g.Gl.assign((size_t)n * gsz, make_double2(0, 0));
        g.Gg.assign((size_t)n * gsz, make_double2(0, 0));
    }
    release(ctx, "gs_V");
    release(ctx, "gs_partbig");
    // (ii) forward meshes of all groups in lockstep
    SilOpts fo = o;
    fo.direction = -1;
    std::vector<GroupSpec> specs;
    std::vector<double2*> ptrs;
    std::vector<int64_t> lds;
    {
        int col = 0;
        for (auto& g : G) {
            specs.push_back(GroupSpec{HModel(g.set.get()), g.sec, col, (int)g.mem.size()});
            col += (int)g.mem.size();
        }
        sil_groups_reserve(ctx, specs, o.m);
    }
    for (int t = 1; t < nt; ++t) {
        specs.clear();
        ptrs.clear();
        lds.clear();
        int col = 0;
        for (auto& g : G) {
            const int n = (int)g.mem.size();
            const int64_t D = g.sec->dim();
            double2* cur = g.Phi + (size_t)t * n * D;
            KGF_HIP(hipMemcpyAsync(cur, cur - (size_t)n * D, sizeof(double2) * (size_t)n * D, hipMemcpyDeviceToDevice,
                                   ctx->stream));
            specs.push_back(GroupSpec{HModel(g.set.get()), g.sec, col, n});
            ptrs.push_back(cur);
            lds.push_back(D);
            col += n;
        }
        for (int r = 0; r < spg; ++r) sil_step_groups(ctx, specs, ptrs, lds, fo);
        progress(ctx, "forward", t, nt - 1);
    }
    // (iii)+(iv) backward sweeps of all groups in lockstep
    SilOpts so = o;
    so.direction = +1;
    for (int spin = 0; spin < 2; ++spin) {
        std::vector<int> loc;
        for (int a = 0; a < norb; ++a)
            if ((orbs[a] & 1) == spin) loc.push_back(a);
        const int na = (int)loc.size();
        if (!na) continue;
        DevBuf gidx;
        upload_ints(ctx, gidx, loc);
        for (int dagger = 0; dagger < 2; ++dagger) {
            const size_t rsz = (size_t)nt * nt * na * na;
            size_t per_j = 0;    // device bytes per source time (all groups' columns with their Krylov slots)
            for (size_t gi = 0; gi < G.size(); ++gi) {
                LockGroup& g = G[gi];
                g.tgt = shifted(ctx, g.sec, spin, dagger ? +1 : -1);
                if (!g.tgt || g.tgt->dim() == 0) {
                    g.tgt.reset();
                    continue;
                }
                per_j += sizeof(double2) * (size_t)(o.m + 1) * na * g.mem.size() * g.tgt->dim();
                g.raw = static_cast<double2*>(workspace(ctx, "lneq_raw" + std::to_string(gi),
                                                        sizeof(double2) * rsz * g.mem.size()));
                KGF_HIP(hipMemsetAsync(g.raw, 0, sizeof(double2) * rsz * g.mem.size(), ctx->stream));
            }
            if (per_j == 0) continue;
            int jchunk = nt;
            if (batch > 0) {
                size_t cols_per_j = 0;
                for (auto& g : G)
                    if (g.tgt) cols_per_j += (size_t)na * g.mem.size();
                jchunk = std::max<int>(1, (int)(batch / std::max<size_t>(cols_per_j, 1)));
            } else {
                size_t free_b = 0, total_b = 0;
                KGF_HIP(hipMemGetInfo(&free_b, &total_b));
                jchunk = (int)std::max<size_t>(1, (size_t)(0.8 * (double)free_b) / per_j);
            }
            jchunk = std::min(jchunk, nt);
            release(ctx, "sg_X");
            for (size_t gi = 0; gi < G.size(); ++gi) {
                LockGroup& g = G[gi];
                if (!g.tgt) continue;
                const size_t n = g.mem.size();
                const int64_t Dt = g.tgt->dim();
                const size_t maxcols = (size_t)jchunk * na * n;
                ensure_device_fits(sizeof(double2) * maxcols * Dt, "batched four-step sweep block");
                g.S = static_cast<double2*>(workspace(ctx, "lneq_cols" + std::to_string(gi),
                                                      sizeof(double2) * maxcols * Dt));
                g.Lb = static_cast<double2*>(workspace(ctx, "lneq_left" + std::to_string(gi),
                                                       sizeof(double2) * (size_t)na * n * Dt));
                g.tmp = static_cast<double2*>(workspace(ctx, "lneq_tmp" + std::to_string(gi),
                                                        sizeof(double2) * (size_t)na * jchunk * na));
            }
            {   // the widest step of the sweep: a full chunk of every group
                specs.clear();
                int col = 0;
                for (auto& g : G) {
                    if (!g.tgt) continue;
                    const int nc = jchunk * na * (int)g.mem.size();
                    specs.push_back(GroupSpec{HModel(g.set.get()), g.tgt.get(), col, nc});
                    col += nc;
                }
                sil_groups_reserve(ctx, specs, o.m);
            }
            const int64_t ss = (int64_t)na * na * nt, sb = (int64_t)na * nt, sa = nt, sj = 1;
            for (int jhi = nt - 1; jhi >= 0; jhi -= jchunk) {
                const int jlo = std::max(0, jhi - jchunk + 1);
                int ncur = 0;   // columns per member; column (r, member) at S + (r * n + member) * Dt
                for (int s2 = jhi; s2 >= 0; --s2) {
                    const bool inject = s2 >= jlo;
                    for (auto& g : G) {
                        if (!g.tgt) continue;
                        const int n = (int)g.mem.size();
                        const int64_t D = g.sec->dim(), Dt = g.tgt->dim();
                        const double2* phi = g.Phi + (size_t)s2 * n * D;
                        if (inject)
                            for (int q = 0; q < na; ++q)
                                apply_c(ctx, g.sec, g.tgt.get(), orbs[loc[q]], dagger, phi,
                                        g.S + (size_t)(ncur + q) * n * Dt, n, D, Dt);
                        for (int q = 0; q < na; ++q)
                            apply_c(ctx, g.sec, g.tgt.get(), orbs[loc[q]], dagger, phi, g.Lb + (size_t)q * n * Dt, n,
                                    D, Dt);
                        const int nc = ncur + (inject ? na : 0);
                        for (int k = 0; k < n; ++k) {
                            block_dots(ctx, g.Lb + (size_t)k * Dt, (int64_t)n * Dt, na, g.S + (size_t)k * Dt,
                                       (int64_t)n * Dt, nc, Dt, g.tmp, nc);
                            place(ctx, g.tmp, na, na, nc, jhi, g.raw + (size_t)k * rsz, s2 * ss, sb, sa, sj);
                        }
                    }
                    if (inject) ncur += na;
                    if (s2 > 0) {
                        specs.clear();
                        ptrs.clear();
                        lds.clear();
                        int col = 0;
                        for (auto& g : G) {
                            if (!g.tgt) continue;
                            const int nc = ncur * (int)g.mem.size();
                            specs.push_back(GroupSpec{HModel(g.set.get()), g.tgt.get(), col, nc});
                            ptrs.push_back(g.S);
                            lds.push_back(g.tgt->dim());
                            col += nc;
                        }
                        for (int r = 0; r < spg; ++r) sil_step_groups(ctx, specs, ptrs, lds, so);
                    }
                    progress(ctx, dagger ? "batch_sweep_greater" : "batch_sweep_lesser", jhi - s2 + 1, jhi + 1);
                }
            }
            for (size_t gi = 0; gi < G.size(); ++gi) {
                LockGroup& g = G[gi];
                if (!g.tgt) continue;
                const int n = (int)g.mem.size();
                double2* Gdev = static_cast<double2*>(workspace(ctx, "mneq_G", sizeof(double2) * gsz * n));
                KGF_HIP(hipMemsetAsync(Gdev, 0, sizeof(double2) * gsz * n, ctx->stream));
                const int64_t total = (int64_t)nt * nt * na * na;
                for (int k = 0; k < n; ++k) {
                    hipLaunchKernelGGL(k_store_neq, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)),
                                       dim3(kThreads), 0, ctx->stream, g.raw + (size_t)k * rsz, ss, sb, sa, sj, nt, na,
                                       gidx.as<int>(), norb, dagger, 1, Gdev + (size_t)k * gsz);
                    check_launch("k_store_neq");
                }
                std::vector<double2> h((size_t)n * gsz);
                KGF_HIP(hipMemcpyAsync(h.data(), Gdev, sizeof(double2) * h.size(), hipMemcpyDeviceToHost,
                                       ctx->stream));
                sync(ctx);
                std::vector<double2>& dst = dagger ? g.Gg : g.Gl;
                for (size_t e = 0; e < h.size(); ++e)
                    if (h[e].x != 0.0 || h[e].y != 0.0) dst[e] = h[e];
            }
            for (size_t gi = 0; gi < G.size(); ++gi)
                for (const char* nm : {"lneq_cols", "lneq_left", "lneq_tmp"})
                    release(ctx, (std::string(nm) + std::to_string(gi)).c_str());
            release(ctx, "sg_X");
        }
    }
    for (auto& g : G) {
        const int n = (int)g.mem.size();
        for (int k = 0; k < n; ++k) {
            if (Gl_host) std::copy(g.Gl.begin() + (size_t)k * gsz, g.Gl.begin() + (size_t)(k + 1) * gsz,
                                   Gl_host + (size_t)g.mem[k] * gsz);
            if (Gg_host) std::copy(g.Gg.begin() + (size_t)k * gsz, g.Gg.begin() + (size_t)(k + 1) * gsz,
                                   Gg_host + (size_t)g.mem[k] * gsz);
        }
    }
    for (size_t gi = 0; gi < G.size(); ++gi)
        for (const char* nm : {"lneq_phi", "lneq_raw"}) release(ctx, (std::string(nm) + std::to_string(gi)).c_str());
    for (const char* nm : {"mneq_G", "sg_part", "sg_scal"}) release(ctx, nm);
}

static void greens_neq_multi_groups(kgf_ctx* ctx, int ninst, kgf_model* const* Hi, kgf_model* const* Hf,
                                    const kgf_sector* const* secs, const double2* const* v0, const kgf_gs_opts* gso,
                                    const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o, int batch,
                                    double2* Gl_host, double2* Gg_host, double* E0_host);

// Instances whose sector has at most this many states run their groups in
// lockstep (their per-group launches are too small to fill the GPU); larger
// ones run group by group with the single-group kernels, whose arguments the
// hardware preloads (the grouped kernels read a descriptor per block, about
// 5% slower per launch when the launch alone fills the GPU).
constexpr int64_t kLockstepMaxDim = int64_t(1) << 17;

void greens_neq_multi(kgf_ctx* ctx, int ninst, kgf_model* const* Hi, kgf_model* const* Hf,
                      const kgf_sector* const* secs, const double2* const* v0, const kgf_gs_opts* gso,
                      const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o, int batch, double2* Gl_host,
                      double2* Gg_host, double* E0_host) {
    TraceRange range_("kgf four-step, many instances");
    std::vector<int> small, large;
    for (int i = 0; i < ninst; ++i) (secs[i]->dim() <= kLockstepMaxDim ? small : large).push_back(i);
    std::vector<kgf_model*> small_h;
    std::vector<const kgf_sector*> small_s;
    for (int i : small) {
        small_h.push_back(Hf[i]);
        small_s.push_back(secs[i]);
    }
    if (!ctx->lockstep || small.size() < 2 ||
        !lockstep_possible(ctx, (int)small.size(), small_h.data(), small_s.data(), o)) {
        greens_neq_multi_groups(ctx, ninst, Hi, Hf, secs, v0, gso, orbs, norb, nt, spg, o, batch, Gl_host, Gg_host,
                                E0_host);
        return;
    }
    const size_t gsz = (size_t)nt * nt * norb * norb;
    for (int part = 0; part < 2; ++part) {
        const std::vector<int>& idx = part == 0 ? small : large;
        if (idx.empty()) continue;
        const int n = (int)idx.size();
        std::vector<kgf_model*> hi(n), hf(n);
        std::vector<const kgf_sector*> sc(n);
        std::vector<const double2*> v(n);
        std::vector<double2> gl(Gl_host ? (size_t)n * gsz : 0), gg(Gg_host ? (size_t)n * gsz : 0);
        std::vector<double> e0(n);
        for (int k = 0; k < n; ++k) {
            hi[k] = Hi[idx[k]];
            hf[k] = Hf[idx[k]];
            sc[k] = secs[idx[k]];
            v[k] = v0[idx[k]];
        }
        if (part == 0)
            greens_neq_multi_lockstep(ctx, n, hi.data(), hf.data(), sc.data(), v.data(), gso, orbs, norb, nt, spg, o,
                                      batch, Gl_host ? gl.data() : nullptr, Gg_host ? gg.data() : nullptr, e0.data());
        else
            greens_neq_multi_groups(ctx, n, hi.data(), hf.data(), sc.data(), v.data(), gso, orbs, norb, nt, spg, o,
                                    batch, Gl_host ? gl.data() : nullptr, Gg_host ? gg.data() : nullptr, e0.data());
        for (int k = 0; k < n; ++k) {
            E0_host[idx[k]] = e0[k];
            if (Gl_host) std::copy(gl.begin() + (size_t)k * gsz, gl.begin() + (size_t)(k + 1) * gsz,
                                   Gl_host + (size_t)idx[k] * gsz);
            if (Gg_host) std::copy(gg.begin() + (size_t)k * gsz, gg.begin() + (size_t)(k + 1) * gsz,
                                   Gg_host + (size_t)idx[k] * gsz);
        }
    }
}

static void greens_neq_multi_groups(kgf_ctx* ctx, int ninst, kgf_model* const* Hi, kgf_model* const* Hf,
                                    const kgf_sector* const* secs, const double2* const* v0, const kgf_gs_opts* gso,
                                    const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o, int batch,
                                    double2* Gl_host, double2* Gg_host, double* E0_host) {
    std::vector<int> done(ninst, 0);
    const size_t gsz = (size_t)nt * nt * norb * norb;
    for (int i0 = 0; i0 < ninst; ++i0) {
        if (done[i0]) continue;
        std::vector<int> mem;
        for (int i = i0; i < ninst; ++i)
            if (!done[i] && secs[i]->L == secs[i0]->L && secs[i]->n_up == secs[i0]->n_up &&
                secs[i]->n_dn == secs[i0]->n_dn && same_topology(Hf[i], Hf[i0])) {
                mem.push_back(i);
                done[i] = 1;
            }
        const int n = (int)mem.size();
        const kgf_sector* sec = secs[i0];
        const int64_t D = sec->dim();
        const size_t vb = sizeof(double2) * (size_t)D;
        ModelSet Sf;
        for (int i : mem) Sf.models.push_back(Hf[i]);
        model_set_init(ctx, Sf);
        // (i) ground states, (ii) forward meshes Phi[k][member]
        ensure_device_fits(vb * (size_t)nt * n, "batched four-step forward meshes");
        double2* Phi = static_cast<double2*>(workspace(ctx, "mneq_phi", vb * (size_t)nt * n));
        for (int k = 0; k < n; ++k) {
            GsResult gs = ground_state(ctx, Hi[mem[k]], sec, v0[mem[k]], Phi + (size_t)k * D, gso->tol, gso->max_iter,
                                       gso->check_every, gso->reorth);
            KGF_REQUIRE(gs.converged, KGF_ENOCONV, "batched four-step: a ground state of H_ini did not converge");
            require_unique_ground_state(ctx, Hi[mem[k]], sec, Phi + (size_t)k * D, gso, "batched four-step");
            E0_host[mem[k]] = gs.E0;
            progress(ctx, "ground_states", k + 1, n);
        }
        release(ctx, "gs_V");
        release(ctx, "gs_partbig");
        SilOpts fo = o;
        fo.direction = -1;
        for (int t = 1; t < nt; ++t) {
            double2* cur = Phi + (size_t)t * n * D;
            KGF_HIP(hipMemcpyAsync(cur, cur - (size_t)n * D, vb * n, hipMemcpyDeviceToDevice, ctx->stream));
            sil_propagate(ctx, HModel(&Sf), sec, cur, n, D, spg, fo);
            progress(ctx, "forward", t, nt - 1);
        }
        auto phi = [&](int t) { return Phi + (size_t)t * n * D; };
        std::vector<double2> Gl((size_t)n * gsz, make_double2(0, 0)), Gg((size_t)n * gsz, make_double2(0, 0));
        SilOpts so = o;
        so.direction = +1;
        for (int spin = 0; spin < 2; ++spin) {
            std::vector<int> loc;
            for (int a = 0; a < norb; ++a)
                if ((orbs[a] & 1) == spin) loc.push_back(a);
            const int na = (int)loc.size();
            if (!na) continue;
            DevBuf gidx;
            upload_ints(ctx, gidx, loc);
            for (int dagger = 0; dagger < 2; ++dagger) {
                auto tgt = shifted(ctx, sec, spin, dagger ? +1 : -1);
                if (!tgt || tgt->dim() == 0) continue;
                const int64_t Dt = tgt->dim();
                const size_t rsz = (size_t)nt * nt * na * na;
                double2* raw = static_cast<double2*>(workspace(ctx, "mneq_raw", sizeof(double2) * rsz * n));
                KGF_HIP(hipMemsetAsync(raw, 0, sizeof(double2) * rsz * n, ctx->stream));
                const size_t per_col = sizeof(double2) * (size_t)(o.m + 1) * Dt;
                int Bcols = batch;
                if (Bcols <= 0) {
                    size_t free_b = 0, total_b = 0;
                    KGF_HIP(hipMemGetInfo(&free_b, &total_b));
                    Bcols = (int)std::max<size_t>(1, (size_t)(0.8 * (double)free_b) / per_col);
                }
                const int jchunk = std::min(nt, std::max(1, Bcols / (na * n)));
                const int maxcols = jchunk * na * n;
                release(ctx, "sil_X");
                sil_reserve(ctx, tgt.get(), maxcols, o.m, o.reorth);
                ensure_device_fits(sizeof(double2) * (size_t)maxcols * Dt, "batched four-step sweep block");
                double2* S = static_cast<double2*>(workspace(ctx, "mneq_cols", sizeof(double2) * (size_t)maxcols * Dt));
                double2* Lb = static_cast<double2*>(workspace(ctx, "mneq_left", sizeof(double2) * (size_t)na * n * Dt));
                double2* tmp = static_cast<double2*>(workspace(ctx, "mneq_tmp", sizeof(double2) * (size_t)na * jchunk * na));
                const int64_t ss = (int64_t)na * na * nt, sb = (int64_t)na * nt, sa = nt, sj = 1;
                for (int jhi = nt - 1; jhi >= 0; jhi -= jchunk) {
                    const int jlo = std::max(0, jhi - jchunk + 1);
                    int ncur = 0;   // columns per member; column (r, member) at S + (r * n + member) * Dt
                    for (int s2 = jhi; s2 >= 0; --s2) {
                        if (s2 >= jlo) {
                            for (int q = 0; q < na; ++q)
                                apply_c(ctx, sec, tgt.get(), orbs[loc[q]], dagger, phi(s2),
                                        S + (size_t)(ncur + q) * n * Dt, n, D, Dt);
                            ncur += na;
                        }
                        for (int q = 0; q < na; ++q)
                            apply_c(ctx, sec, tgt.get(), orbs[loc[q]], dagger, phi(s2), Lb + (size_t)q * n * Dt, n, D,
                                    Dt);
                        for (int k = 0; k < n; ++k) {
                            block_dots(ctx, Lb + (size_t)k * Dt, (int64_t)n * Dt, na, S + (size_t)k * Dt,
                                       (int64_t)n * Dt, ncur, Dt, tmp, ncur);
                            place(ctx, tmp, na, na, ncur, jhi, raw + (size_t)k * rsz, s2 * ss, sb, sa, sj);
                        }
                        if (s2 > 0) sil_propagate(ctx, HModel(&Sf), tgt.get(), S, ncur * n, Dt, spg, so);
                        progress(ctx, dagger ? "batch_sweep_greater" : "batch_sweep_lesser", jhi - s2 + 1, jhi + 1);
                    }
                }
                double2* Gdev = static_cast<double2*>(workspace(ctx, "mneq_G", sizeof(double2) * gsz * n));
                KGF_HIP(hipMemsetAsync(Gdev, 0, sizeof(double2) * gsz * n, ctx->stream));
                const int64_t total = (int64_t)nt * nt * na * na;
                for (int k = 0; k < n; ++k) {
                    hipLaunchKernelGGL(k_store_neq, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)),
                                       dim3(kThreads), 0, ctx->stream, raw + (size_t)k * rsz, ss, sb, sa, sj, nt, na,
                                       gidx.as<int>(), norb, dagger, 1, Gdev + (size_t)k * gsz);
                    check_launch("k_store_neq");
                }
                std::vector<double2> h((size_t)n * gsz);
                KGF_HIP(hipMemcpyAsync(h.data(), Gdev, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
                sync(ctx);
                // only the entries of this spin group were written (the rest are zero)
                std::vector<double2>& dst = dagger ? Gg : Gl;
                for (size_t e = 0; e < h.size(); ++e)
                    if (h[e].x != 0.0 || h[e].y != 0.0) dst[e] = h[e];
            }
        }
        for (int k = 0; k < n; ++k) {
            if (Gl_host) std::copy(Gl.begin() + (size_t)k * gsz, Gl.begin() + (size_t)(k + 1) * gsz,
                                   Gl_host + (size_t)mem[k] * gsz);
            if (Gg_host) std::copy(Gg.begin() + (size_t)k * gsz, Gg.begin() + (size_t)(k + 1) * gsz,
                                   Gg_host + (size_t)mem[k] * gsz);
        }
        for (const char* nm : {"mneq_phi", "mneq_cols", "mneq_left", "mneq_raw", "mneq_G", "sil_X"}) release(ctx, nm);
    }
}

// Four-step with a driven final Hamiltonian H(t) = sum_j f_j(t) H_j (the
// commutator-free integrator of driven.hip; steps of o.dt from t = 0, spg per
// mesh interval).  Without time-translation invariance the sweep carries
// X_{a,j}(s) = U(t_j, t_s)^+ c_a Phi_j: from t_s to t_{s-1} each column takes
// the adjoint stage exponentials of the steps in between, last step first and
// B_2 before B_1.  U(t_s, 0) U(t_j, 0)^+ = U(t_j, t_s)^+ for the product of
// steps, so <c_b Phi_s | X_{a,j}(s)> = <Psi_b(t_s)|Psi_a(t_j)> as in the
// plain schedule.  `work` takes every stage's parameters in turn.
void greens_neq_driven(kgf_ctx* ctx, kgf_model* Hi, kgf_model* work, const kgf_sector* sec, const double2* v0,
                       const kgf_gs_opts* gso, const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o,
                       int batch, const DriveTable& drv, double2* Gl_host, double2* Gg_host, double* E0_host) {
    const int64_t D = sec->dim();
    const size_t vb = sizeof(double2) * (size_t)D;
    const size_t gsz = (size_t)nt * nt * norb * norb;
    ensure_device_fits(vb * (size_t)nt, "driven four-step forward mesh");
    double2* Phi = static_cast<double2*>(workspace(ctx, "dneq_phi", vb * (size_t)nt));
    GsResult gs = ground_state(ctx, Hi, sec, v0, Phi, gso->tol, gso->max_iter, gso->check_every, gso->reorth);
    KGF_REQUIRE(gs.converged, KGF_ENOCONV, "driven four-step: the ground state of H_ini did not converge");
    require_unique_ground_state(ctx, Hi, sec, Phi, gso, "driven four-step");
    *E0_host = gs.E0;
    release(ctx, "gs_V");
    release(ctx, "gs_partbig");
    SilOpts fo = o;
    fo.direction = -1;
    for (int t = 1; t < nt; ++t) {
        double2* cur = Phi + (size_t)t * D;
        KGF_HIP(hipMemcpyAsync(cur, cur - D, vb, hipMemcpyDeviceToDevice, ctx->stream));
        for (int n = (t - 1) * spg; n < t * spg; ++n)
            for (int stage = 0; stage < 2; ++stage) {
                driven_stage(work, drv, n, stage);
                sil_propagate(ctx, work, sec, cur, 1, D, 1, fo);
            }
        progress(ctx, "driven_forward", t, nt - 1);
    }
    auto phi = [&](int t) { return Phi + (size_t)t * D; };
    std::vector<double2> Gl(gsz, make_double2(0, 0)), Gg(gsz, make_double2(0, 0));
    SilOpts so = o;
    so.direction = +1;
    for (int spin = 0; spin < 2; ++spin) {
        std::vector<int> loc;
        for (int a = 0; a < norb; ++a)
            if ((orbs[a] & 1) == spin) loc.push_back(a);
        const int na = (int)loc.size();
        if (!na) continue;
        DevBuf gidx;
        upload_ints(ctx, gidx, loc);
        for (int dagger = 0; dagger < 2; ++dagger) {
            auto tgt = shifted(ctx, sec, spin, dagger ? +1 : -1);
            if (!tgt || tgt->dim() == 0) continue;
            const int64_t Dt = tgt->dim();
            const size_t rsz = (size_t)nt * nt * na * na;
            double2* raw = static_cast<double2*>(workspace(ctx, "dneq_raw", sizeof(double2) * rsz));
            KGF_HIP(hipMemsetAsync(raw, 0, sizeof(double2) * rsz, ctx->stream));
            const size_t per_col = sizeof(double2) * (size_t)(o.m + 1) * Dt;
            int Bcols = batch;
            if (Bcols <= 0) {
                size_t free_b = 0, total_b = 0;
                KGF_HIP(hipMemGetInfo(&free_b, &total_b));
                Bcols = (int)std::max<size_t>(1, (size_t)(0.8 * (double)free_b) / per_col);
            }
            const int jchunk = std::min(nt, std::max(1, Bcols / na));
            const int maxcols = jchunk * na;
            release(ctx, "sil_X");
            sil_reserve(ctx, tgt.get(), maxcols, o.m, o.reorth);
            ensure_device_fits(sizeof(double2) * (size_t)maxcols * Dt, "driven four-step sweep block");
            double2* S = static_cast<double2*>(workspace(ctx, "dneq_cols", sizeof(double2) * (size_t)maxcols * Dt));
            double2* Lb = static_cast<double2*>(workspace(ctx, "dneq_left", sizeof(double2) * (size_t)na * Dt));
            double2* tmp = static_cast<double2*>(workspace(ctx, "dneq_tmp", sizeof(double2) * (size_t)na * maxcols));
            const int64_t ss = (int64_t)na * na * nt, sb = (int64_t)na * nt, sa = nt, sj = 1;
            for (int jhi = nt - 1; jhi >= 0; jhi -= jchunk) {
                const int jlo = std::max(0, jhi - jchunk + 1);
                int ncur = 0;   // column r at S + r * Dt: orbital r % na injected at t_{jhi - r / na}
                for (int s2 = jhi; s2 >= 0; --s2) {
                    if (s2 >= jlo) {
                        for (int q = 0; q < na; ++q)
                            apply_c(ctx, sec, tgt.get(), orbs[loc[q]], dagger, phi(s2), S + (size_t)(ncur + q) * Dt,
                                    1, D, Dt);
                        ncur += na;
                    }
                    for (int q = 0; q < na; ++q)
                        apply_c(ctx, sec, tgt.get(), orbs[loc[q]], dagger, phi(s2), Lb + (size_t)q * Dt, 1, D, Dt);
                    block_dots(ctx, Lb, Dt, na, S, Dt, ncur, Dt, tmp, ncur);
                    place(ctx, tmp, na, na, ncur, jhi, raw, s2 * ss, sb, sa, sj);
                    if (s2 > 0)
                        for (int n = s2 * spg - 1; n >= (s2 - 1) * spg; --n)
                            for (int stage = 1; stage >= 0; --stage) {
                                driven_stage(work, drv, n, stage);
                                sil_propagate(ctx, work, tgt.get(), S, ncur, Dt, 1, so);
                            }
                    progress(ctx, dagger ? "driven_sweep_greater" : "driven_sweep_lesser", jhi - s2 + 1, jhi + 1);
                }
            }
            double2* Gdev = static_cast<double2*>(workspace(ctx, "dneq_G", sizeof(double2) * gsz));
            KGF_HIP(hipMemsetAsync(Gdev, 0, sizeof(double2) * gsz, ctx->stream));
            const int64_t total = (int64_t)nt * nt * na * na;
            hipLaunchKernelGGL(k_store_neq, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)),
                               dim3(kThreads), 0, ctx->stream, raw, ss, sb, sa, sj, nt, na, gidx.as<int>(), norb,
                               dagger, 1, Gdev);
            check_launch("k_store_neq");
            std::vector<double2> h(gsz);
            KGF_HIP(hipMemcpyAsync(h.data(), Gdev, sizeof(double2) * gsz, hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            // only the entries of this spin group were written (the rest are zero)
            std::vector<double2>& dst = dagger ? Gg : Gl;
            for (size_t e = 0; e < gsz; ++e)
                if (h[e].x != 0.0 || h[e].y != 0.0) dst[e] = h[e];
        }
    }
    if (Gl_host) std::copy(Gl.begin(), Gl.end(), Gl_host);
    if (Gg_host) std::copy(Gg.begin(), Gg.end(), Gg_host);
    for (const char* nm : {"dneq_phi", "dneq_cols", "dneq_left", "dneq_tmp", "dneq_raw", "dneq_G", "sil_X"})
        release(ctx, nm);
}

// Four-time two-particle functions (the outlook's higher-order Green's
// functions): chi_abcd(t1,t2,t3,t4) = <0| O1_a(t1) O2_b(t2) O3_c(t3) O4_d(t4) |0>,
// O = c or c+ (two of each), as the scalar product of the two-time states
// O2_b(t2)^+ O1_a(t1)^+ |0> and O3_c(t3) O4_d(t4) |0>.  A two-time state
// o_x(s) o_y(u)|0> = e^{iHs} o_x e^{-iH(s-u)} o_y Phi(u), Phi(u) = e^{-iHu}|0>:
// per spin class (spin of x, spin of y), o_y Phi(u) is carried through the
// mesh in its sector (forward from u, then backward from u), o_x applied at
// every mesh time s; the resulting columns, laid out with s slowest, go back
// to t = 0 in one sweep (the columns with s >= k form a contiguous tail that
// takes one mesh interval at step k).  chi is the Gram matrix between bra and
// ket classes that end in the same sector.  host_chi:
// [nt][nt][nt][nt][norb][norb][norb][norb], zero where the spins do not match.
struct TwoTimeClass {
    int sx, sy, nx, ny;
    std::unique_ptr<kgf_sector> s2;
    double2* Z = nullptr;
};

void greens2_neq(kgf_ctx* ctx, kgf_model* Hi, kgf_model* H, const kgf_sector* sec, const double2* v0,
                 const kgf_gs_opts* gso, const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o,
                 const int dag[4], double2* chi_host, double* E0_host) {
    const int64_t D = sec->dim();
    const size_t vb = sizeof(double2) * (size_t)D;
    ensure_device_fits(vb * (size_t)nt, "four-time function: forward mesh");
    double2* Phi = static_cast<double2*>(workspace(ctx, "g2_phi", vb * (size_t)nt));
    GsResult gs = ground_state(ctx, Hi, sec, v0, Phi, gso->tol, gso->max_iter, gso->check_every, gso->reorth);
    KGF_REQUIRE(gs.converged, KGF_ENOCONV, "four-time function: the ground state of H_ini did not converge");
    require_unique_ground_state(ctx, Hi, sec, Phi, gso, "four-time function");
    *E0_host = gs.E0;
    release(ctx, "gs_V");
    release(ctx, "gs_partbig");
    SilOpts fo = o, bo = o;
    fo.direction = -1;
    bo.direction = +1;
    for (int t = 1; t < nt; ++t) {
        double2* cur = Phi + (size_t)t * D;
        KGF_HIP(hipMemcpyAsync(cur, cur - D, vb, hipMemcpyDeviceToDevice, ctx->stream));
        sil_propagate(ctx, H, sec, cur, 1, D, spg, fo);
    }
    std::vector<int> by_spin[2];
    for (int a = 0; a < norb; ++a) by_spin[orbs[a] & 1].push_back(a);
    const int64_t total_chi = (int64_t)nt * nt * nt * nt * norb * norb * norb * norb;
    std::fill(chi_host, chi_host + total_chi, make_double2(0.0, 0.0));

    // all states o_x(t_s) o_y(t_u)|0> (o = c+ where the flag is set), class by class
    auto family = [&](int dx, int dy, const char* tag) {
        std::vector<TwoTimeClass> cls;
        for (int sx = 0; sx < 2; ++sx)
            for (int sy = 0; sy < 2; ++sy) {
                const int nx = (int)by_spin[sx].size(), ny = (int)by_spin[sy].size();
                if (!nx || !ny) continue;
                auto s1 = shifted(ctx, sec, sy, dy ? +1 : -1);
                if (!s1 || s1->dim() == 0) continue;
                auto s2 = shifted(ctx, s1.get(), sx, dx ? +1 : -1);
                if (!s2 || s2->dim() == 0) continue;
                const int64_t D1 = s1->dim(), D2 = s2->dim();
                const int blk = nt * nx * ny;                       // columns per mesh time s
                const size_t zb = sizeof(double2) * (size_t)nt * blk * D2;
                ensure_device_fits(zb + 2 * sizeof(double2) * (size_t)ny * D1, "four-time function: two-time states");
                const std::string zname = std::string(tag) + std::to_string(2 * sx + sy);
                double2* Z = static_cast<double2*>(workspace(ctx, zname, zb));
                double2* W = static_cast<double2*>(workspace(ctx, "g2_W", sizeof(double2) * (size_t)ny * D1));
                double2* W0 = static_cast<double2*>(workspace(ctx, "g2_W0", sizeof(double2) * (size_t)ny * D1));
                // column ((s * nt + u) * nx + i) * ny + j  <->  o_{x_i}(t_s) o_{y_j}(t_u)|0>
                auto emit = [&](int s_, int u_) {
                    for (int i = 0; i < nx; ++i)
                        apply_c(ctx, s1.get(), s2.get(), orbs[by_spin[sx][i]], dx, W,
                                Z + (size_t)(((int64_t)s_ * nt + u_) * nx + i) * ny * D2, ny, D1, D2);
                };
                for (int u = 0; u < nt; ++u) {
                    for (int j = 0; j < ny; ++j)
                        apply_c(ctx, sec, s1.get(), orbs[by_spin[sy][j]], dy, Phi + (size_t)u * D,
                                W0 + (size_t)j * D1, 1, D, D1);
                    KGF_HIP(hipMemcpyAsync(W, W0, sizeof(double2) * (size_t)ny * D1, hipMemcpyDeviceToDevice,
                                           ctx->stream));
                    emit(u, u);
                    for (int s_ = u + 1; s_ < nt; ++s_) {              // e^{-iH(t_s - t_u)}, s > u
                        sil_propagate(ctx, H, s1.get(), W, ny, D1, spg, fo);
                        emit(s_, u);
                    }
                    KGF_HIP(hipMemcpyAsync(W, W0, sizeof(double2) * (size_t)ny * D1, hipMemcpyDeviceToDevice,
                                           ctx->stream));
                    for (int s_ = u - 1; s_ >= 0; --s_) {              // s < u
                        sil_propagate(ctx, H, s1.get(), W, ny, D1, spg, bo);
                        emit(s_, u);
                    }
                    progress(ctx, "four_time_states", u + 1, nt);
                }
                for (int k = nt - 1; k >= 1; --k)                       // e^{iH t_s}: columns s >= k, one interval
                    sil_propagate(ctx, H, s2.get(), Z + (size_t)k * blk * D2, (nt - k) * blk, D2, spg, bo);
                TwoTimeClass c;
                c.sx = sx;
                c.sy = sy;
                c.nx = nx;
                c.ny = ny;
                c.s2 = std::move(s2);
                c.Z = Z;
                cls.push_back(std::move(c));
            }
        return cls;
    };
    // kets O3_c(t3) O4_d(t4)|0>; bras O2_b(t2)^+ O1_a(t1)^+ |0>
    std::vector<TwoTimeClass> kets = family(dag[2], dag[3], "g2k_Z");
    std::vector<TwoTimeClass> bras_own;
    const bool same = (1 - dag[1]) == dag[2] && (1 - dag[0]) == dag[3];
    if (!same) bras_own = family(1 - dag[1], 1 - dag[0], "g2b_Z");
    const std::vector<TwoTimeClass>& bras = same ? kets : bras_own;
    for (const TwoTimeClass& bra : bras)
        for (const TwoTimeClass& ket : kets) {
            if (bra.s2->n_up != ket.s2->n_up || bra.s2->n_dn != ket.s2->n_dn) continue;
            const int nl = nt * nt * bra.nx * bra.ny, nr = nt * nt * ket.nx * ket.ny;
            double2* gram = static_cast<double2*>(workspace(ctx, "g2_gram", sizeof(double2) * (size_t)nl * nr));
            block_dots(ctx, bra.Z, bra.s2->dim(), nl, ket.Z, ket.s2->dim(), nr, bra.s2->dim(), gram, nr);
            std::vector<double2> h((size_t)nl * nr);
            KGF_HIP(hipMemcpyAsync(h.data(), gram, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            // bra column (s = t2, u = t1, x = b, y = a); ket column (s = t3, u = t4, x = c, y = d)
            for (int l = 0; l < nl; ++l) {
                const int jb = l % bra.ny, ib = (l / bra.ny) % bra.nx;
                const int u1 = (l / (bra.ny * bra.nx)) % nt, s2_ = l / (bra.ny * bra.nx * nt);
                const int A = by_spin[bra.sy][jb], B = by_spin[bra.sx][ib];
                for (int r = 0; r < nr; ++r) {
                    const int jk = r % ket.ny, ik = (r / ket.ny) % ket.nx;
                    const int u4 = (r / (ket.ny * ket.nx)) % nt, s3 = r / (ket.ny * ket.nx * nt);
                    const int Cc = by_spin[ket.sx][ik], Dd = by_spin[ket.sy][jk];
                    const int64_t e =
                        ((((((((int64_t)u1 * nt + s2_) * nt + s3) * nt + u4) * norb + A) * norb + B) * norb + Cc) *
                             norb +
                         Dd);
                    chi_host[e] = h[(size_t)l * nr + r];
                }
            }
        }
    for (const char* nm : {"g2_phi", "g2_W", "g2_W0", "g2_gram", "g2k_Z0", "g2k_Z1", "g2k_Z2", "g2k_Z3", "g2b_Z0",
                           "g2b_Z1", "g2b_Z2", "g2b_Z3", "sil_X"})
        release(ctx, nm);
}

}  // namespace kgf

using namespace kgf;

extern "C" int kgf_greens_neq(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                              const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                              int nt, int steps_per_grid, const kgf_prop_opts* opts, int schedule, int batch,
                              int ntau, int tau_steps_per_grid, double dtau, kgf_c128* host_G_lesser,
                              kgf_c128* host_G_greater, kgf_c128* host_G_matsubara, kgf_c128* host_G_mixed,
                              kgf_c128* host_G_mixed_left, double* host_E0, kgf_c128* psi0_out) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(ctx && H_ini && H && sector && gs_opts && v0 && host_orbs && host_E0, KGF_EINVAL,
                    "kgf_greens_neq: NULL argument");
        KGF_REQUIRE(H_ini->L == sector->L && H->L == sector->L, KGF_EINVAL,
                    "kgf_greens_neq: models and sector differ in L");
        KGF_REQUIRE(sector->dim() > 0, KGF_EINVAL, "kgf_greens_neq: empty sector");
        kgf::check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && (schedule == 0 || schedule == 1) && batch >= 0,
                    KGF_EINVAL, "kgf_greens_neq: bad sizes");
        KGF_REQUIRE(ntau >= 0 && (ntau == 0 || (tau_steps_per_grid >= 1 && std::isfinite(dtau) && dtau >= 0.0)),
                    KGF_EINVAL, "kgf_greens_neq: bad Matsubara mesh");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        kgf::gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens_neq: bad ground-state options");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sector->L, KGF_EINVAL,
                        "kgf_greens_neq: orbital out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        NeqArgs A;
        A.H_ini = const_cast<kgf_model*>(H_ini);
        A.H = const_cast<kgf_model*>(H);
        A.sec = sector;
        A.orbs = host_orbs;
        A.norb = n_orb;
        A.nt = nt;
        A.spg = steps_per_grid;
        A.o = kgf::to_sil_opts(opts);
        A.schedule = schedule;
        A.batch = batch;
        A.ntau = ntau;
        A.tspg = tau_steps_per_grid;
        A.dtau = dtau;
        greens_neq(ctx, A, reinterpret_cast<const double2*>(v0), gs_opts, host_E0,
                   reinterpret_cast<double2*>(psi0_out), reinterpret_cast<double2*>(host_G_lesser),
                   reinterpret_cast<double2*>(host_G_greater), reinterpret_cast<double2*>(host_G_matsubara),
                   reinterpret_cast<double2*>(host_G_mixed), reinterpret_cast<double2*>(host_G_mixed_left));
    });
}

// Step-wise four-step run (sweep schedule): steps (i) and (ii) at creation,
// then steps (iii) and (iv) one mesh interval per kgf_neq_run_advance call,
// through the same SweepBranch code as kgf_greens_neq (bitwise the same G).
// The run keeps its own workspaces: the context's are swapped out while a
// run call executes, so other calls on the context in between do not touch
// the run's forward mesh or sweep block.
struct kgf_neq_run {
    kgf_ctx* ctx = nullptr;
    std::map<std::string, std::unique_ptr<kgf::DevBuf>> ws;
    std::vector<int32_t> orbs;
    kgf::NeqArgs A;
    kgf::PhiMesh Phi;
    double E0 = 0.0;
    std::vector<std::pair<int, int>> branches;    // (spin, dagger), kgf_greens_neq's order
    std::vector<std::vector<int>> locs;           // orbital indices of each branch's spin
    size_t next = 0;
    std::unique_ptr<kgf::SweepBranch> cur;
    double2* Gl = nullptr;
    double2* Gg = nullptr;
    int64_t vector_steps = 0;
    bool done = false;
    bool touched = false;   // advanced or restored since creation
};

namespace {
struct RunWorkspaces {
    kgf_ctx* ctx;
    std::map<std::string, std::unique_ptr<kgf::DevBuf>>& own;
    RunWorkspaces(kgf_ctx* c, std::map<std::string, std::unique_ptr<kgf::DevBuf>>& w) : ctx(c), own(w) {
        std::swap(ctx->ws, own);
    }
    ~RunWorkspaces() { std::swap(ctx->ws, own); }
};

// begin the next branch whose target sector is not empty; false when none is left
bool run_next_branch(kgf_neq_run* r) {
    while (r->next < r->branches.size()) {
        const auto [spin, dagger] = r->branches[r->next];
        const auto& loc = r->locs[r->next];
        ++r->next;
        std::unique_ptr<kgf::SweepBranch> br(new kgf::SweepBranch());
        if (br->begin(r->ctx, r->A, loc, spin, dagger, nullptr)) {
            r->cur = std::move(br);
            return true;
        }
    }
    r->cur.reset();
    return false;
}
}  // namespace

extern "C" int kgf_neq_run_create(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                                  const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                                  int nt, int steps_per_grid, const kgf_prop_opts* opts, int batch,
                                  kgf_neq_run** out, double* host_E0) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(ctx && H_ini && H && sector && gs_opts && v0 && host_orbs && out && host_E0, KGF_EINVAL,
                    "kgf_neq_run_create: NULL argument");
        KGF_REQUIRE(H_ini->L == sector->L && H->L == sector->L, KGF_EINVAL,
                    "kgf_neq_run_create: models and sector differ in L");
        KGF_REQUIRE(sector->dim() > 0, KGF_EINVAL, "kgf_neq_run_create: empty sector");
        kgf::check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && batch >= 0, KGF_EINVAL,
                    "kgf_neq_run_create: bad sizes");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        kgf::gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_neq_run_create: bad ground-state options");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sector->L, KGF_EINVAL,
                        "kgf_neq_run_create: orbital out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        std::unique_ptr<kgf_neq_run> r(new kgf_neq_run());
        r->ctx = ctx;
        r->orbs.assign(host_orbs, host_orbs + n_orb);
        kgf::NeqArgs& A = r->A;
        A.H_ini = const_cast<kgf_model*>(H_ini);
        A.H = const_cast<kgf_model*>(H);
        A.sec = sector;
        A.orbs = r->orbs.data();
        A.norb = n_orb;
        A.nt = nt;
        A.spg = steps_per_grid;
        A.o = kgf::to_sil_opts(opts);
        A.schedule = 1;
        A.batch = batch;
        A.ntau = 0;
        A.tspg = 1;
        A.dtau = 0.0;
        RunWorkspaces guard(ctx, r->ws);
        kgf::neq_forward(ctx, A, reinterpret_cast<const double2*>(v0), gs_opts, &r->E0, nullptr, r->Phi);
        const size_t gsz = sizeof(double2) * (size_t)nt * nt * n_orb * n_orb;
        r->Gl = static_cast<double2*>(kgf::workspace(ctx, "run_Gl", gsz));
        r->Gg = static_cast<double2*>(kgf::workspace(ctx, "run_Gg", gsz));
        KGF_HIP(hipMemsetAsync(r->Gl, 0, gsz, ctx->stream));
        KGF_HIP(hipMemsetAsync(r->Gg, 0, gsz, ctx->stream));
        for (int spin = 0; spin < 2; ++spin) {
            std::vector<int> loc;
            for (int a = 0; a < n_orb; ++a)
                if ((host_orbs[a] & 1) == spin) loc.push_back(a);
            if (loc.empty()) continue;
            for (int dagger = 0; dagger < 2; ++dagger) {
                r->branches.push_back({spin, dagger});
                r->locs.push_back(loc);
            }
        }
        r->done = !run_next_branch(r.get());
        kgf::sync(ctx);
        *host_E0 = r->E0;
        *out = r.release();
    });
}

extern "C" int kgf_neq_run_advance(kgf_neq_run* r, int n_intervals, kgf_neq_run_info* host_info) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(r && n_intervals >= 0, KGF_EINVAL, "kgf_neq_run_advance: bad argument");
        kgf_ctx* ctx = r->ctx;
        KGF_HIP(hipSetDevice(ctx->device));
        RunWorkspaces guard(ctx, r->ws);
        int64_t steps = 0;
        int ran = 0, width = 0;
        while (ran < n_intervals && !r->done) {
            width = r->cur->next_width();
            steps += r->cur->interval(r->Phi);
            ++ran;
            if (r->cur->finished()) {
                const int dagger = r->cur->dagger;
                r->cur->finish(dagger ? r->Gg : r->Gl, nullptr);
                kgf::sync(ctx);
                r->done = !run_next_branch(r);
            }
        }
        r->vector_steps += steps;
        if (ran > 0) r->touched = true;
        if (host_info) {
            host_info->intervals = ran;
            host_info->vector_steps = steps;
            host_info->width = width;
            host_info->done = r->done ? 1 : 0;
            host_info->next_width = r->done ? 0 : r->cur->next_width();
            host_info->next_mesh_index = r->done ? -1 : r->cur->next_s();
            host_info->chunk_width = r->done ? 0 : r->cur->chunk_width();
            host_info->branch = r->done ? -1 : (int)r->next - 1;
            host_info->total_vector_steps = r->vector_steps;
            host_info->chunk_start = (r->done || !r->cur->in_chunk) ? 1 : 0;
        }
    });
}

namespace {
// Byte image of a run between chunks: header, G^<, G^> as accumulated so
// far, and the current branch's placed dot products.
struct RunImageHeader {
    uint64_t magic;          // kRunImageMagic
    int64_t D;               // sector dimension
    int32_t nt, norb;
    int32_t branch;          // index into kgf_neq_run::branches of the current branch, -1 when done
    int32_t jhi, jchunk, na; // next chunk's top mesh index, chunk length, orbitals of the branch
    int64_t vector_steps;
    double E0;
};
constexpr uint64_t kRunImageMagic = 0x6b67666e72756e31ULL;   // "kgfnrun1"

size_t run_image_bytes(const kgf_neq_run* r) {
    const size_t g = sizeof(double2) * (size_t)r->A.nt * r->A.nt * r->A.norb * r->A.norb;
    size_t raw = 0;
    if (!r->done && r->cur) raw = sizeof(double2) * (size_t)r->A.nt * r->A.nt * r->cur->na * r->cur->na;
    return sizeof(RunImageHeader) + 2 * g + raw;
}
}  // namespace

extern "C" int kgf_neq_run_checkpoint(kgf_neq_run* r, void* host_buf, size_t bytes, size_t* host_bytes_needed) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(r, KGF_EINVAL, "kgf_neq_run_checkpoint: NULL run");
        const size_t need = run_image_bytes(r);
        if (host_bytes_needed) *host_bytes_needed = need;
        if (!host_buf) return;   // size query
        KGF_REQUIRE(bytes >= need, KGF_EINVAL, "kgf_neq_run_checkpoint: buffer too small");
        KGF_REQUIRE(r->done || !r->cur->in_chunk, KGF_EINVAL,
                    "kgf_neq_run_checkpoint: the run is inside a chunk (checkpoint where next_width == chunk_width)");
        kgf_ctx* ctx = r->ctx;
        KGF_HIP(hipSetDevice(ctx->device));
        RunImageHeader h{};
        h.magic = kRunImageMagic;
        h.D = r->A.sec->dim();
        h.nt = r->A.nt;
        h.norb = r->A.norb;
        h.branch = r->done ? -1 : (int32_t)r->next - 1;
        h.jhi = r->done ? -1 : r->cur->jhi;
        h.jchunk = r->done ? 0 : r->cur->jchunk;
        h.na = r->done ? 0 : r->cur->na;
        h.vector_steps = r->vector_steps;
        h.E0 = r->E0;
        char* out = static_cast<char*>(host_buf);
        std::memcpy(out, &h, sizeof h);
        const size_t g = sizeof(double2) * (size_t)r->A.nt * r->A.nt * r->A.norb * r->A.norb;
        char* p = out + sizeof h;
        KGF_HIP(hipMemcpyAsync(p, r->Gl, g, hipMemcpyDeviceToHost, ctx->stream));
        KGF_HIP(hipMemcpyAsync(p + g, r->Gg, g, hipMemcpyDeviceToHost, ctx->stream));
        if (!r->done)
            KGF_HIP(hipMemcpyAsync(p + 2 * g, r->cur->raw, need - sizeof h - 2 * g, hipMemcpyDeviceToHost,
                                   ctx->stream));
        kgf::sync(ctx);
    });
}

extern "C" int kgf_neq_run_restore(kgf_neq_run* r, const void* host_buf, size_t bytes) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(r && host_buf, KGF_EINVAL, "kgf_neq_run_restore: NULL argument");
        KGF_REQUIRE(bytes >= sizeof(RunImageHeader), KGF_EINVAL, "kgf_neq_run_restore: image too short");
        RunImageHeader h;
        std::memcpy(&h, host_buf, sizeof h);
        KGF_REQUIRE(h.magic == kRunImageMagic, KGF_EINVAL, "kgf_neq_run_restore: not a run image");
        KGF_REQUIRE(h.D == r->A.sec->dim() && h.nt == r->A.nt && h.norb == r->A.norb, KGF_EINVAL,
                    "kgf_neq_run_restore: image of a run with other sizes");
        KGF_REQUIRE(std::abs(h.E0 - r->E0) <= 1e-12 * std::max(1.0, std::abs(r->E0)), KGF_EINVAL,
                    "kgf_neq_run_restore: image of a run with another ground state");
        KGF_REQUIRE(!r->touched, KGF_EINVAL,
                    "kgf_neq_run_restore: the run has already advanced or been restored (restore into a new run)");
        KGF_REQUIRE(h.branch >= -1 && h.branch < (int32_t)r->branches.size(), KGF_EINVAL,
                    "kgf_neq_run_restore: branch out of range");
        const size_t g = sizeof(double2) * (size_t)r->A.nt * r->A.nt * r->A.norb * r->A.norb;
        const size_t raw = h.branch >= 0 ? sizeof(double2) * (size_t)r->A.nt * r->A.nt * h.na * h.na : 0;
        KGF_REQUIRE(bytes >= sizeof h + 2 * g + raw, KGF_EINVAL, "kgf_neq_run_restore: image too short");
        kgf_ctx* ctx = r->ctx;
        KGF_HIP(hipSetDevice(ctx->device));
        RunWorkspaces guard(ctx, r->ws);
        const char* p = static_cast<const char*>(host_buf) + sizeof h;
        KGF_HIP(hipMemcpyAsync(r->Gl, p, g, hipMemcpyHostToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(r->Gg, p + g, g, hipMemcpyHostToDevice, ctx->stream));
        if (h.branch < 0) {
            r->cur.reset();
            r->next = r->branches.size();
            r->done = true;
        } else {
            // begin the saved branch with the saved chunk length, so that its
            // blocks (and their rounding) are those of the run that was saved
            KGF_REQUIRE(h.na == (int32_t)r->locs[(size_t)h.branch].size() && h.jchunk >= 1 &&
                            h.jchunk <= r->A.nt && h.jhi >= 0 && h.jhi < r->A.nt,
                        KGF_EINVAL, "kgf_neq_run_restore: inconsistent branch state");
            r->cur.reset();
            r->next = (size_t)h.branch;
            const int batch = r->A.batch;
            r->A.batch = h.jchunk * h.na;
            const bool ok = run_next_branch(r);
            r->A.batch = batch;
            KGF_REQUIRE(ok && (int32_t)r->next - 1 == h.branch, KGF_EINVAL,
                        "kgf_neq_run_restore: the saved branch has no work in this run");
            r->cur->jhi = h.jhi;
            KGF_HIP(hipMemcpyAsync(r->cur->raw, p + 2 * g, raw, hipMemcpyHostToDevice, ctx->stream));
        }
        r->vector_steps = h.vector_steps;
        r->touched = true;
        kgf::sync(ctx);
    });
}

extern "C" int kgf_neq_run_result(kgf_neq_run* r, kgf_c128* host_G_lesser, kgf_c128* host_G_greater) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(r, KGF_EINVAL, "kgf_neq_run_result: NULL run");
        KGF_REQUIRE(r->done, KGF_EINVAL, "kgf_neq_run_result: the run has intervals left");
        kgf_ctx* ctx = r->ctx;
        KGF_HIP(hipSetDevice(ctx->device));
        const size_t gsz = sizeof(double2) * (size_t)r->A.nt * r->A.nt * r->A.norb * r->A.norb;
        if (host_G_lesser) KGF_HIP(hipMemcpyAsync(host_G_lesser, r->Gl, gsz, hipMemcpyDeviceToHost, ctx->stream));
        if (host_G_greater) KGF_HIP(hipMemcpyAsync(host_G_greater, r->Gg, gsz, hipMemcpyDeviceToHost, ctx->stream));
        kgf::sync(ctx);
    });
}

extern "C" void kgf_neq_run_destroy(kgf_neq_run* r) {
    if (!r) return;
    (void)hipSetDevice(r->ctx->device);
    (void)hipStreamSynchronize(r->ctx->stream);
    delete r;
}

extern "C" int kgf_greens_neq_multi(kgf_ctx* ctx, int n_inst, const kgf_model* const* H_ini,
                                    const kgf_model* const* H, const kgf_sector* const* sectors,
                                    const kgf_c128* const* v0, const kgf_gs_opts* gs_opts, const int32_t* host_orbs,
                                    int n_orb, int nt, int steps_per_grid, const kgf_prop_opts* opts, int batch,
                                    kgf_c128* host_G_lesser, kgf_c128* host_G_greater, double* host_E0) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(ctx && n_inst >= 1 && H_ini && H && sectors && v0 && gs_opts && host_orbs && host_E0, KGF_EINVAL,
                    "kgf_greens_neq_multi: NULL argument");
        kgf::check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && batch >= 0, KGF_EINVAL,
                    "kgf_greens_neq_multi: bad sizes");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        kgf::gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens_neq_multi: bad ground-state options");
        for (int i = 0; i < n_inst; ++i) {
            KGF_REQUIRE(H_ini[i] && H[i] && sectors[i] && v0[i], KGF_EINVAL, "kgf_greens_neq_multi: NULL instance");
            KGF_REQUIRE(H_ini[i]->L == sectors[i]->L && H[i]->L == sectors[i]->L && sectors[i]->dim() > 0,
                        KGF_EINVAL, "kgf_greens_neq_multi: model / sector mismatch or empty sector");
            for (int a = 0; a < n_orb; ++a)
                KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sectors[i]->L, KGF_EINVAL,
                            "kgf_greens_neq_multi: orbital out of range");
        }
        KGF_HIP(hipSetDevice(ctx->device));
        greens_neq_multi(ctx, n_inst, const_cast<kgf_model* const*>(H_ini), const_cast<kgf_model* const*>(H), sectors,
                         reinterpret_cast<const double2* const*>(v0), gs_opts, host_orbs, n_orb, nt, steps_per_grid,
                         kgf::to_sil_opts(opts), batch, reinterpret_cast<double2*>(host_G_lesser),
                         reinterpret_cast<double2*>(host_G_greater), host_E0);
    });
}

extern "C" int kgf_greens_neq_driven(kgf_ctx* ctx, const kgf_model* H_ini, kgf_model* work,
                                     const kgf_sector* sector, const kgf_gs_opts* gs_opts, const kgf_c128* v0,
                                     const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                                     const kgf_prop_opts* opts, int batch, int n_terms, const double* host_theta,
                                     const double* host_f, kgf_c128* host_G_lesser, kgf_c128* host_G_greater,
                                     double* host_E0) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(ctx && H_ini && work && sector && gs_opts && v0 && host_orbs && host_E0 && host_theta && host_f,
                    KGF_EINVAL, "kgf_greens_neq_driven: NULL argument");
        KGF_REQUIRE(H_ini != work, KGF_EINVAL, "kgf_greens_neq_driven: work must not be H_ini");
        KGF_REQUIRE(H_ini->L == sector->L && work->L == sector->L, KGF_EINVAL,
                    "kgf_greens_neq_driven: models and sector differ in L");
        KGF_REQUIRE(sector->dim() > 0, KGF_EINVAL, "kgf_greens_neq_driven: empty sector");
        kgf::check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && batch >= 0 && n_terms >= 1, KGF_EINVAL,
                    "kgf_greens_neq_driven: bad sizes");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        kgf::gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens_neq_driven: bad ground-state options");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sector->L, KGF_EINVAL,
                        "kgf_greens_neq_driven: orbital out of range");
        const int nth = kgf::n_theta(work);
        const int64_t nsteps = (int64_t)(nt - 1) * steps_per_grid;
        for (int64_t i = 0; i < (int64_t)n_terms * nth; ++i)
            KGF_REQUIRE(std::isfinite(host_theta[i]), KGF_EINVAL, "kgf_greens_neq_driven: non-finite theta");
        for (int64_t i = 0; i < nsteps * 2 * n_terms; ++i)
            KGF_REQUIRE(std::isfinite(host_f[i]), KGF_EINVAL, "kgf_greens_neq_driven: non-finite drive value");
        KGF_HIP(hipSetDevice(ctx->device));
        greens_neq_driven(ctx, const_cast<kgf_model*>(H_ini), work, sector, reinterpret_cast<const double2*>(v0),
                          gs_opts, host_orbs, n_orb, nt, steps_per_grid, kgf::to_sil_opts(opts), batch,
                          kgf::DriveTable{n_terms, host_theta, host_f}, reinterpret_cast<double2*>(host_G_lesser),
                          reinterpret_cast<double2*>(host_G_greater), host_E0);
    });
}

extern "C" int kgf_greens2_neq(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                               const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                               int nt, int steps_per_grid, const kgf_prop_opts* opts, int pattern,
                               kgf_c128* host_chi, double* host_E0) {
    return kgf::abi_guard([&] {
        KGF_REQUIRE(ctx && H_ini && H && sector && gs_opts && v0 && host_orbs && host_chi && host_E0, KGF_EINVAL,
                    "kgf_greens2_neq: NULL argument");
        KGF_REQUIRE(H_ini->L == sector->L && H->L == sector->L, KGF_EINVAL,
                    "kgf_greens2_neq: models and sector differ in L");
        KGF_REQUIRE(sector->dim() > 0, KGF_EINVAL, "kgf_greens2_neq: empty sector");
        kgf::check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1, KGF_EINVAL, "kgf_greens2_neq: bad sizes");
        const double n4 = (double)nt * nt * nt * nt * n_orb * n_orb * n_orb * n_orb;
        KGF_REQUIRE(n4 <= (double)(1 << 28), KGF_EUNSUPPORTED, "kgf_greens2_neq: nt^4 n_orb^4 above 2^28");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        kgf::gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens2_neq: bad ground-state options");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sector->L, KGF_EINVAL,
                        "kgf_greens2_neq: orbital out of range");
        KGF_REQUIRE(pattern >= 0 && pattern < 16 && __builtin_popcount((unsigned)pattern) == 2, KGF_EINVAL,
                    "kgf_greens2_neq: pattern must hold two c+ and two c");
        const int dag[4] = {(pattern >> 3) & 1, (pattern >> 2) & 1, (pattern >> 1) & 1, pattern & 1};
        KGF_HIP(hipSetDevice(ctx->device));
        greens2_neq(ctx, const_cast<kgf_model*>(H_ini), const_cast<kgf_model*>(H), sector,
                    reinterpret_cast<const double2*>(v0), gs_opts, host_orbs, n_orb, nt, steps_per_grid,
                    kgf::to_sil_opts(opts), dag, reinterpret_cast<double2*>(host_chi), host_E0);
    });
}
