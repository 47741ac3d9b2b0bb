// Reverse mode (adjoint) of the short-iterative-Lanczos propagation and of
// the four-step nonequilibrium Green's function (Sec. 4), with respect to
// the parameters theta = (t_b, eps_up_i, eps_dn_i, U_i) of H and of H_ini.
//
// A real loss L with dL = Re sum conj(W) dG (W = the cotangent of G) is
// propagated backwards.  Cotangents are psi_bar = dL/d(psi*), so that
// dL = 2 Re <psi_bar| d psi>.
//   * One step psi_{n+1} = exp(delta i H dt) psi_n (delta = -1 forward,
//     +1 backward; each step is numerically exact in its Krylov space):
//       psi_bar_n = exp(-delta i H dt) psi_bar_{n+1},
//       dL/dtheta += 2 Re[ delta i int_0^dt <lam(s)| dH/dtheta |psi(s)> ds ],
//       psi(s) = exp(delta i H s) psi_n, lam(s) = exp(-delta i H (dt - s)) psi_bar_{n+1}
//     (derivative of the exponential under the integral, Duhamel form).  The
//     integral uses Gauss-Legendre nodes; the states at the nodes come from
//     the step's own Krylov spaces (the fine-grid evaluation of Eq. (udelta)).
//   * c_a and c+_a are parameter free; their adjoints are c+_a and c_a.
//   * Ground state: d|0> = -(H_ini - E0)^+ (1 - P0) dH_ini |0> gives
//     dL/dtheta_ini = -2 Re <mu| dH_ini/dtheta |0>, (H_ini - E0) mu = (1 - P0) 0_bar,
//     mu orthogonal to |0> (projected conjugate gradients).
#include <algorithm>
#include <cmath>
#include <complex>

#include "kgf_internal.h"

namespace kgf {

namespace {

using cplx = std::complex<double>;

// Gauss-Legendre nodes x_q and weights w_q on [-1, 1] (Newton on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pq = q == 1 ? z : p1;
            const double pqm1 = q == 1 ? 1.0 : p0;
            const double dp = q * (z * pq - pqm1) / (z * z - 1.0);
            const double dz = pq / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= q; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double pq = q == 1 ? z : p1;
        const double pqm1 = q == 1 ? 1.0 : p0;
        const double dp = q * (z * pq - pqm1) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

__global__ void k_axpy(double2* __restrict__ y, const double2* __restrict__ x, double ar, double ai, int64_t D) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = x[i];
        double2 b = y[i];
        b.x += ar * a.x - ai * a.y;
        b.y += ar * a.y + ai * a.x;
        y[i] = b;
    }
}

// p = r + beta p
__global__ void k_xpby(double2* __restrict__ p, const double2* __restrict__ r, double beta, int64_t D) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = r[i];
        const double2 b = p[i];
        p[i] = make_double2(a.x + beta * b.x, a.y + beta * b.y);
    }
}

// out[y] = sum_z C[y][z] in[z] for ny outputs (dense complex combination)
__global__ __launch_bounds__(kThreads) void k_lincomb(const double2* __restrict__ in, int64_t in_col, int nz,
                                                      const double2* __restrict__ C, double2* __restrict__ out,
                                                      int64_t out_col, int64_t D) {
    const int y = blockIdx.y;
    const double2* c = C + (int64_t)y * nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int z = 0; z < nz; ++z) {
            const double2 a = in[z * in_col + i];
            const double2 h = c[z];
            re = fma(h.x, a.x, fma(-h.y, a.y, re));
            im = fma(h.x, a.y, fma(h.y, a.x, im));
        }
        out[y * out_col + i] = make_double2(re, im);
    }
}

int grid_for(int64_t D) {
    int64_t b = (D + kThreads * 4 - 1) / (kThreads * 4);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

void axpy(kgf_ctx* ctx, double2* y, const double2* x, cplx a, int64_t D) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(D)), dim3(kThreads), 0, ctx->stream, y, x, a.real(), a.imag(), D);
    check_launch("k_axpy");
}

cplx dot(kgf_ctx* ctx, const double2* a, const double2* b, int64_t D) {
    double2* d = static_cast<double2*>(workspace(ctx, "adj_dot", sizeof(double2)));
    block_dots(ctx, a, D, 1, b, D, 1, D, d);
    double2 h;
    KGF_HIP(hipMemcpyAsync(&h, d, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    return cplx(h.x, h.y);
}

std::unique_ptr<kgf_sector> adj_sector(kgf_ctx* ctx, int L, int nu, int nd) {
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

}  // namespace

// One adjoint step of psi_{n+1} = exp(delta i H dt) psi_n (see the file header)
// for nm members at once (member c uses the Hamiltonian of launch column c mod
// nm: a single model, or a ModelSet).  psi: members at stride psi_ld; lam: on
// entry psi_bar_{n+1}, on return psi_bar_n (stride lam_ld); g (device) gets
// member j's gradient at g + j * gstride.
void sil_adjoint_step(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int nm, const double2* psi, int64_t psi_ld,
                      double2* lam, int64_t lam_ld, double dt, int delta, const SilOpts& o, int nq, double* g,
                      int gstride) {
    const int64_t D = sec->dim();
    const int m = o.m;
    const size_t vb = sizeof(double2) * (size_t)D;
    double2* pair = static_cast<double2*>(workspace(ctx, "adj_pair", vb * 2 * nm));   // [psi_j][lam_j]
    for (int j = 0; j < nm; ++j) {
        KGF_HIP(hipMemcpyAsync(pair + (size_t)j * D, psi + j * psi_ld, vb, hipMemcpyDeviceToDevice, ctx->stream));
        KGF_HIP(hipMemcpyAsync(pair + (size_t)(nm + j) * D, lam + j * lam_ld, vb, hipMemcpyDeviceToDevice,
                               ctx->stream));
    }
    sil_build(ctx, model, sec, pair, 2 * nm, D, o);
    std::vector<double> xq, wq;
    gauss_legendre(nq, xq, wq);
    const int per = 2 * nq + 1;
    const int nreq = per * nm;
    std::vector<int> col(nreq), dir(nreq);
    std::vector<double> tt(nreq);
    for (int j = 0; j < nm; ++j) {
        const int r0 = j * per;
        for (int q = 0; q < nq; ++q) {
            const double s = 0.5 * dt * (1.0 + xq[q]);
            col[r0 + q] = j, dir[r0 + q] = delta, tt[r0 + q] = s;                        // psi(s)
            col[r0 + nq + q] = nm + j, dir[r0 + nq + q] = -delta, tt[r0 + nq + q] = dt - s;  // lam(s)
        }
        col[r0 + 2 * nq] = nm + j, dir[r0 + 2 * nq] = -delta, tt[r0 + 2 * nq] = dt;     // new cotangent
    }
    double2* coef = static_cast<double2*>(workspace(ctx, "adj_coef", sizeof(double2) * nreq * m));
    sil_coefs(ctx, m, nreq, col.data(), tt.data(), dir.data(), 0.0, coef, m);
    // per member: nq psi nodes, nq lam nodes, the new cotangent (one slot)
    const int slots = 2 * nq + 1;
    double2* nodes = static_cast<double2*>(workspace(ctx, "adj_nodes", vb * slots * nm));
    std::vector<double2> om(nq);
    for (int q = 0; q < nq; ++q) {
        // 2 Re[delta i (dt/2) w_q <lam|dH|psi>]  ->  weight delta i dt w_q
        om[q] = make_double2(0.0, delta * dt * wq[q]);
    }
    for (int j = 0; j < nm; ++j) {
        const double2* cj = coef + (size_t)j * per * m;
        double2* nj = nodes + (size_t)j * slots * D;
        sil_combine_multi(ctx, sec, pair, D, 2 * nm, m, j, cj, m, nq, nj, D);
        // lam nodes and the new cotangent in one pass over the lam basis
        sil_combine_multi(ctx, sec, pair, D, 2 * nm, m, nm + j, cj + (size_t)nq * m, m, nq + 1, nj + (size_t)nq * D, D);
        KGF_HIP(hipMemcpyAsync(lam + j * lam_ld, nj + (size_t)2 * nq * D, vb, hipMemcpyDeviceToDevice, ctx->stream));
        // dH/dtheta depends on the bond topology only, shared by all members
        dH_expect(ctx, model.m, sec, nj + (size_t)nq * D, D, nj, D, nq, om.data(), g + (size_t)j * gstride);
    }
}

// Adjoint of nm chains x_{n+1} = exp(delta i H dt) x_n, n < nsteps, from x_0
// (members at stride x_ld).  lam: in the cotangents of x_nsteps, out those of
// x_0 (stride lam_ld).  The states x_n are needed in reverse order.  They are
// stored whole when they take at most 30% of free device memory (unless
// ctx->adj_every forces checkpoints); otherwise every K-th state is kept and
// each segment of K states is recomputed forward from its checkpoint just
// before its adjoint steps (recomputed states are bitwise the stored ones).
void chain_adjoint(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int nm, const double2* x0, int64_t x_ld,
                   int nsteps, double dt, int delta, const SilOpts& o, int nq, double2* lam, int64_t lam_ld, double* g,
                   int gstride) {
    if (nsteps <= 0) return;
    const int64_t D = sec->dim();
    const size_t vb = sizeof(double2) * (size_t)D * nm;   // one state of all members
    const int64_t sd = D * nm;
    SilOpts so = o;
    so.dt = dt;
    so.direction = delta;
    auto load = [&](double2* dst) {
        for (int j = 0; j < nm; ++j)
            KGF_HIP(hipMemcpyAsync(dst + (size_t)j * D, x0 + j * x_ld, sizeof(double2) * D, hipMemcpyDeviceToDevice,
                                   ctx->stream));
    };
    int K = ctx->adj_every;
    if (K <= 0) {
        size_t free_b = 0, total_b = 0;
        KGF_HIP(hipMemGetInfo(&free_b, &total_b));
        K = nsteps;
        if ((double)vb * nsteps > 0.30 * (double)free_b)
            for (K = 1; K < nsteps; ++K)
                if ((double)vb * ((nsteps + K - 1) / K + K) <= 0.30 * (double)free_b) break;
    }
    K = std::max(1, std::min(K, nsteps));
    if (K >= nsteps) {
        ensure_device_fits(vb * (size_t)nsteps, "adjoint chain states");
        double2* S = static_cast<double2*>(workspace(ctx, "adj_chain", vb * (size_t)nsteps));
        load(S);
        for (int n = 1; n < nsteps; ++n) {
            KGF_HIP(hipMemcpyAsync(S + (size_t)n * sd, S + (size_t)(n - 1) * sd, vb, hipMemcpyDeviceToDevice,
                                   ctx->stream));
            sil_propagate(ctx, model, sec, S + (size_t)n * sd, nm, D, 1, so);
        }
        for (int n = nsteps - 1; n >= 0; --n)
            sil_adjoint_step(ctx, model, sec, nm, S + (size_t)n * sd, D, lam, lam_ld, dt, delta, o, nq, g, gstride);
        return;
    }
    // checkpoints C[c] = x_{cK}, then segments of K states
    const int ncp = (nsteps + K - 1) / K;
    ensure_device_fits(vb * (size_t)(ncp + K), "adjoint chain checkpoints");
    double2* Cp = static_cast<double2*>(workspace(ctx, "adj_chain", vb * (size_t)(ncp + K)));
    double2* Sg = Cp + (size_t)ncp * sd;
    load(Cp);
    load(Sg);
    for (int n = 1; n < nsteps; ++n) {
        sil_propagate(ctx, model, sec, Sg, nm, D, 1, so);
        if (n % K == 0)
            KGF_HIP(hipMemcpyAsync(Cp + (size_t)(n / K) * sd, Sg, vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    for (int c = ncp - 1; c >= 0; --c) {
        const int n0 = c * K, n1 = std::min(nsteps, n0 + K);
        KGF_HIP(hipMemcpyAsync(Sg, Cp + (size_t)c * sd, vb, hipMemcpyDeviceToDevice, ctx->stream));
        for (int n = n0 + 1; n < n1; ++n) {
            double2* x = Sg + (size_t)(n - n0) * sd;
            KGF_HIP(hipMemcpyAsync(x, x - sd, vb, hipMemcpyDeviceToDevice, ctx->stream));
            sil_propagate(ctx, model, sec, x, nm, D, 1, so);
        }
        for (int n = n1 - 1; n >= n0; --n)
            sil_adjoint_step(ctx, model, sec, nm, Sg + (size_t)(n - n0) * sd, D, lam, lam_ld, dt, delta, o, nq, g,
                             gstride);
    }
}

// (H - E0) mu = (1 - P0) r, mu orthogonal to psi0 (unit norm), by projected CG.
// *converged: the residual reached tol (false after maxit iterations or a
// non-positive curvature p^T (H - E0) p).
static int projected_cg(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0, double E0,
                        const double2* rhs, double2* mu, double tol, int maxit, bool* converged) {
    *converged = false;
    const int64_t D = sec->dim();
    double2* r = static_cast<double2*>(workspace(ctx, "cg_r", sizeof(double2) * D));
    double2* p = static_cast<double2*>(workspace(ctx, "cg_p", sizeof(double2) * D));
    double2* Ap = static_cast<double2*>(workspace(ctx, "cg_Ap", sizeof(double2) * D));
    KGF_HIP(hipMemsetAsync(mu, 0, sizeof(double2) * D, ctx->stream));
    KGF_HIP(hipMemcpyAsync(r, rhs, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
    axpy(ctx, r, psi0, -dot(ctx, psi0, r, D), D);
    KGF_HIP(hipMemcpyAsync(p, r, sizeof(double2) * D, hipMemcpyDeviceToDevice, ctx->stream));
    double rr = dot(ctx, r, r, D).real();
    const double bnorm = std::sqrt(rr);
    if (bnorm == 0.0) {
        *converged = true;
        return 0;
    }
    int it = 0;
    for (; it < maxit; ++it) {
        apply_h(ctx, model, sec, p, Ap, 1, D);
        axpy(ctx, Ap, p, cplx(-E0, 0.0), D);
        axpy(ctx, Ap, psi0, -dot(ctx, psi0, Ap, D), D);
        const double pAp = dot(ctx, p, Ap, D).real();
        if (!(pAp > 0.0)) break;
        const double alpha = rr / pAp;
        axpy(ctx, mu, p, cplx(alpha, 0.0), D);
        axpy(ctx, r, Ap, cplx(-alpha, 0.0), D);
        const double rr2 = dot(ctx, r, r, D).real();
        if (std::sqrt(rr2) <= tol * bnorm) {
            ++it;
            *converged = true;
            break;
        }
        hipLaunchKernelGGL(k_xpby, dim3(grid_for(D)), dim3(kThreads), 0, ctx->stream, p, r, rr2 / rr, D);
        check_launch("k_xpby");
        rr = rr2;
    }
    axpy(ctx, mu, psi0, -dot(ctx, psi0, mu, D), D);
    return it;
}

// One instance of a four-step adjoint: its Hamiltonians, start vector,
// cotangents (host, [nt][nt][n_orb][n_orb] or null) and host outputs.
struct VjpMember {
    kgf_model* Hi = nullptr;
    kgf_model* Hf = nullptr;
    const double2* v0 = nullptr;
    const double2* Wl = nullptr;
    const double2* Wg = nullptr;
    double* grad_ini = nullptr;
    double* grad = nullptr;
    double2* Gl = nullptr;
    double2* Gg = nullptr;
    double* E0 = nullptr;
    int* cg_iters = nullptr;
    bool cg_failed = false;
};

struct VjpArgs {
    const kgf_sector* sec;
    const int32_t* orbs;
    int norb, nt, spg;
    SilOpts o;
    int nq;
    double cg_tol;
    int cg_maxit;
};

// Gradient of the four-step G (plain schedule) for nm members with one sector
// and one bond topology of H.  Every propagation, chain adjoint and adjoint
// step runs all members as one batch (column c: member c mod nm); ground
// states, Gram matrices, cotangent combinations and the ground-state solves
// are per member.  Mesh states are stored member-fastest: [state][member][D].
static void four_step_vjp(kgf_ctx* ctx, const VjpArgs& A, const kgf_gs_opts* gso, std::vector<VjpMember>& M) {
    TraceRange range_("kgf four-step adjoint");
    const kgf_sector* sec = A.sec;
    const int nm = (int)M.size();
    const int64_t D = sec->dim();
    const int nt = A.nt, norb = A.norb, L = sec->L;
    const double dt = A.o.dt;
    const size_t vb = sizeof(double2) * (size_t)D;
    ModelSet Sf;
    for (auto& mb : M) Sf.models.push_back(mb.Hf);
    if (nm > 1) model_set_init(ctx, Sf);
    const HModel HF = nm > 1 ? HModel(&Sf) : HModel(M[0].Hf);
    // (i) ground states
    double2* psi0 = static_cast<double2*>(workspace(ctx, "vjp_psi0", vb * nm));
    std::vector<double> E0(nm);
    for (int j = 0; j < nm; ++j) {
        GsResult gs = ground_state(ctx, M[j].Hi, sec, M[j].v0, psi0 + (size_t)j * D, gso->tol, gso->max_iter,
                                   gso->check_every, gso->reorth);
        KGF_REQUIRE(gs.converged, KGF_ENOCONV, "adjoint: ground state of H_ini did not converge");
        require_unique_ground_state(ctx, M[j].Hi, sec, psi0 + (size_t)j * D, gso, "adjoint");
        E0[j] = gs.E0;
        if (M[j].E0) *M[j].E0 = gs.E0;
    }
    ctx->ws.erase("gs_V");
    // (ii) forward mesh Phi[k][member]
    const int64_t sd = D * nm;
    ensure_device_fits(vb * nm * (size_t)2 * nt, "adjoint forward mesh");
    double2* Phi = static_cast<double2*>(workspace(ctx, "vjp_phi", vb * nm * (size_t)nt));
    double2* Phib = static_cast<double2*>(workspace(ctx, "vjp_phibar", vb * nm * (size_t)nt));
    KGF_HIP(hipMemsetAsync(Phib, 0, vb * nm * (size_t)nt, ctx->stream));
    KGF_HIP(hipMemcpyAsync(Phi, psi0, vb * nm, hipMemcpyDeviceToDevice, ctx->stream));
    SilOpts fo = A.o;
    fo.direction = -1;
    for (int k = 1; k < nt; ++k) {
        KGF_HIP(hipMemcpyAsync(Phi + (size_t)k * sd, Phi + (size_t)(k - 1) * sd, vb * nm, hipMemcpyDeviceToDevice,
                               ctx->stream));
        sil_propagate(ctx, HF, sec, Phi + (size_t)k * sd, nm, D, A.spg, fo);
    }
    const int nth = n_theta(M[0].Hf);
    int nthi = 0;
    for (auto& mb : M) nthi = std::max(nthi, n_theta(mb.Hi));
    double* g = static_cast<double*>(workspace(ctx, "vjp_g", sizeof(double) * (size_t)nm * (nth + nthi)));
    double* gi = g + (size_t)nm * nth;
    KGF_HIP(hipMemsetAsync(g, 0, sizeof(double) * (size_t)nm * (nth + nthi), ctx->stream));
    const size_t gsz = (size_t)nt * nt * norb * norb;
    std::vector<double2> Gl(gsz * nm, make_double2(0, 0)), Gg(gsz * nm, make_double2(0, 0));
    auto Widx = [&](int j, int k, int a, int b) { return (((size_t)j * nt + k) * norb + a) * norb + b; };
    SilOpts bo = A.o;
    bo.direction = +1;
    // (iii)+(iv) and their adjoints, per spin group and operator
    for (int spin = 0; spin < 2; ++spin) {
        std::vector<int> loc;
        for (int a = 0; a < norb; ++a)
            if ((A.orbs[a] & 1) == spin) loc.push_back(a);
        const int na = (int)loc.size();
        if (!na) continue;
        for (int dagger = 0; dagger < 2; ++dagger) {
            auto tgt = adj_sector(ctx, L, sec->n_up + (spin == 0 ? (dagger ? 1 : -1) : 0),
                                  sec->n_dn + (spin == 1 ? (dagger ? 1 : -1) : 0));
            if (!tgt || tgt->dim() == 0) continue;
            const int64_t Dt = tgt->dim();
            const int64_t tsd = Dt * nm;
            const int N = na * nt;
            ensure_device_fits(sizeof(double2) * (size_t)2 * N * tsd, "adjoint state mesh");
            double2* Psi = static_cast<double2*>(workspace(ctx, "vjp_psi", sizeof(double2) * (size_t)N * tsd));
            double2* Psib = static_cast<double2*>(workspace(ctx, "vjp_psibar", sizeof(double2) * (size_t)N * tsd));
            for (int q = 0; q < na; ++q)
                for (int k = 0; k < nt; ++k) {
                    double2* x = Psi + ((size_t)q * nt + k) * tsd;
                    apply_c(ctx, sec, tgt.get(), A.orbs[loc[q]], dagger, Phi + (size_t)k * sd, x, nm, D, Dt);
                    if (k > 0) sil_propagate(ctx, HF, tgt.get(), x, nm, Dt, k * A.spg, bo);
                    progress(ctx, dagger ? "adjoint_mesh_greater" : "adjoint_mesh_lesser", (int64_t)q * nt + k + 1, N);
                }
            double2* raw = static_cast<double2*>(workspace(ctx, "vjp_raw", sizeof(double2) * (size_t)N * N));
            double2* Cd = static_cast<double2*>(workspace(ctx, "vjp_C", sizeof(double2) * (size_t)N * N));
            std::vector<double2> rh((size_t)N * N), C((size_t)N * N);
            for (int j = 0; j < nm; ++j) {
                // Gram matrix raw[(b,s)][(a,j)] = <Psi_b(s)|Psi_a(j)> of member j
                block_dots(ctx, Psi + (size_t)j * Dt, tsd, N, Psi + (size_t)j * Dt, tsd, N, Dt, raw);
                KGF_HIP(hipMemcpyAsync(rh.data(), raw, sizeof(double2) * rh.size(), hipMemcpyDeviceToHost,
                                       ctx->stream));
                sync(ctx);
                double2* GlJ = Gl.data() + (size_t)j * gsz;
                double2* GgJ = Gg.data() + (size_t)j * gsz;
                for (int a = 0; a < na; ++a)
                    for (int b = 0; b < na; ++b)
                        for (int jj = 0; jj < nt; ++jj)
                            for (int s2 = 0; s2 < nt; ++s2) {
                                // lesser: G[j][s][A][B] = i <Psi_B(s)|Psi_A(j)>; greater: -i <chi_A(j)|chi_B(s)>
                                const double2 z = rh[((size_t)b * nt + s2) * N + (size_t)a * nt + jj];
                                const double2 zg = rh[((size_t)a * nt + jj) * N + (size_t)b * nt + s2];
                                if (!dagger) GlJ[Widx(jj, s2, loc[a], loc[b])] = make_double2(-z.y, z.x);
                                else GgJ[Widx(jj, s2, loc[a], loc[b])] = make_double2(zg.y, -zg.x);
                            }
                // cotangents of the mesh states: Psi_bar = C Psi (see the file header)
                const double2* W = dagger ? M[j].Wg : M[j].Wl;
                for (int x = 0; x < na; ++x)
                    for (int mm = 0; mm < nt; ++mm)
                        for (int a = 0; a < na; ++a)
                            for (int jj = 0; jj < nt; ++jj) {
                                cplx c(0.0, 0.0);
                                if (W) {
                                    const double2 w1 = W[Widx(jj, mm, loc[a], loc[x])];
                                    const double2 w2 = W[Widx(mm, jj, loc[x], loc[a])];
                                    if (!dagger)   // (i/2)[conj(W[j][m][a][x]) - W[m][j][x][a]]
                                        c = cplx(0.0, 0.5) * (std::conj(cplx(w1.x, w1.y)) - cplx(w2.x, w2.y));
                                    else           // (i/2)[W[j][m][a][x] - conj(W[m][j][x][a])]
                                        c = cplx(0.0, 0.5) * (cplx(w1.x, w1.y) - std::conj(cplx(w2.x, w2.y)));
                                }
                                C[((size_t)x * nt + mm) * N + (size_t)a * nt + jj] = make_double2(c.real(), c.imag());
                            }
                KGF_HIP(hipMemcpy(Cd, C.data(), sizeof(double2) * C.size(), hipMemcpyHostToDevice));
                for (int y0 = 0; y0 < N; y0 += 65535) {
                    const int ny = std::min(N - y0, 65535);
                    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(Dt), ny), dim3(kThreads), 0, ctx->stream,
                                       Psi + (size_t)j * Dt, tsd, N, Cd + (size_t)y0 * N,
                                       Psib + (size_t)y0 * tsd + (size_t)j * Dt, tsd, Dt);
                    check_launch("k_lincomb");
                }
                sync(ctx);   // Cd is reused by the next member
            }
            // back through each chain, then through c_a (adjoint c+_a) or c+_a (adjoint c_a)
            double2* xs = static_cast<double2*>(workspace(ctx, "vjp_x0", sizeof(double2) * (size_t)tsd));
            double2* back = static_cast<double2*>(workspace(ctx, "vjp_back", vb * nm));
            for (int q = 0; q < na; ++q)
                for (int k = 0; k < nt; ++k) {
                    double2* lam = Psib + ((size_t)q * nt + k) * tsd;
                    if (k > 0) {
                        apply_c(ctx, sec, tgt.get(), A.orbs[loc[q]], dagger, Phi + (size_t)k * sd, xs, nm, D, Dt);
                        chain_adjoint(ctx, HF, tgt.get(), nm, xs, Dt, k * A.spg, dt, +1, A.o, A.nq, lam, Dt, g, nth);
                    }
                    apply_c(ctx, tgt.get(), sec, A.orbs[loc[q]], dagger ? 0 : 1, lam, back, nm, Dt, D);
                    axpy(ctx, Phib + (size_t)k * sd, back, cplx(1.0, 0.0), sd);
                    progress(ctx, dagger ? "adjoint_greater" : "adjoint_lesser", (int64_t)q * nt + k + 1, N);
                }
        }
    }
    // adjoint of the forward mesh Phi(t_k) = exp(-iH dt)^(k spg) |0>
    double2* lam = static_cast<double2*>(workspace(ctx, "vjp_lam", vb * nm));
    KGF_HIP(hipMemcpyAsync(lam, Phib + (size_t)(nt - 1) * sd, vb * nm, hipMemcpyDeviceToDevice, ctx->stream));
    for (int k = nt - 1; k >= 1; --k) {
        chain_adjoint(ctx, HF, sec, nm, Phi + (size_t)(k - 1) * sd, D, A.spg, dt, -1, A.o, A.nq, lam, D, g, nth);
        axpy(ctx, lam, Phib + (size_t)(k - 1) * sd, cplx(1.0, 0.0), sd);
        progress(ctx, "adjoint_forward", nt - k, nt - 1);
    }
    // ground states of H_ini
    for (int j = 0; j < nm; ++j) {
        int it = 0;
        if (M[j].Wl || M[j].Wg) {
            double2* mu = static_cast<double2*>(workspace(ctx, "vjp_mu", vb));
            bool conv = false;
            it = projected_cg(ctx, M[j].Hi, sec, psi0 + (size_t)j * D, E0[j], lam + (size_t)j * D, mu, A.cg_tol,
                              A.cg_maxit, &conv);
            M[j].cg_failed = !conv;
            const double2 wm = make_double2(-2.0, 0.0);
            dH_expect(ctx, M[j].Hi, sec, mu, D, psi0 + (size_t)j * D, D, 1, &wm, gi + (size_t)j * nthi);
        }
        if (M[j].cg_iters) *M[j].cg_iters = it;
    }
    std::vector<double> gh((size_t)nm * (nth + nthi));
    KGF_HIP(hipMemcpyAsync(gh.data(), g, sizeof(double) * gh.size(), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    for (int j = 0; j < nm; ++j) {
        if (M[j].grad) std::copy(gh.begin() + (size_t)j * nth, gh.begin() + (size_t)(j + 1) * nth, M[j].grad);
        if (M[j].grad_ini) {
            const double* src = gh.data() + (size_t)nm * nth + (size_t)j * nthi;
            std::copy(src, src + n_theta(M[j].Hi), M[j].grad_ini);
        }
        if (M[j].Gl) std::copy(Gl.begin() + (size_t)j * gsz, Gl.begin() + (size_t)(j + 1) * gsz, M[j].Gl);
        if (M[j].Gg) std::copy(Gg.begin() + (size_t)j * gsz, Gg.begin() + (size_t)(j + 1) * gsz, M[j].Gg);
    }
    for (const char* n : {"vjp_phi", "vjp_phibar", "vjp_psi", "vjp_psibar", "adj_chain", "sil_X", "adj_nodes", "adj_pair"})
        ctx->ws.erase(n);
}

}  // namespace kgf

using namespace kgf;

extern "C" {

int kgf_n_theta(const kgf_model* model) { return model ? kgf::n_theta(model) : KGF_EINVAL; }

int kgf_dH_expect(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector, const kgf_c128* lam,
                  const kgf_c128* psi, int npair, int64_t ld, const kgf_c128* host_w, double* host_grad) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && model && sector && host_grad && host_w, KGF_EINVAL, "kgf_dH_expect: NULL argument");
        KGF_REQUIRE(model->L == sector->L, KGF_EINVAL, "kgf_dH_expect: model and sector L differ");
        KGF_REQUIRE(npair >= 0 && ld >= sector->dim(), KGF_EINVAL, "kgf_dH_expect: bad npair / ld");
        KGF_REQUIRE(npair == 0 || (lam && psi), KGF_EINVAL, "kgf_dH_expect: NULL vector");
        KGF_HIP(hipSetDevice(ctx->device));
        const int nth = n_theta(model);
        double* g = static_cast<double*>(workspace(ctx, "abi_grad", sizeof(double) * nth));
        KGF_HIP(hipMemsetAsync(g, 0, sizeof(double) * nth, ctx->stream));
        if (npair > 0 && sector->dim() > 0)
            dH_expect(ctx, const_cast<kgf_model*>(model), sector, reinterpret_cast<const double2*>(lam), ld,
                      reinterpret_cast<const double2*>(psi), ld, npair, reinterpret_cast<const double2*>(host_w), g);
        KGF_HIP(hipMemcpyAsync(host_grad, g, sizeof(double) * nth, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    });
}

int kgf_propagate_vjp(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector, const kgf_c128* psi0,
                      kgf_c128* lam, int nsteps, const kgf_prop_opts* opts, int quad_nodes, double* host_grad) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && model && sector && psi0 && lam && host_grad, KGF_EINVAL,
                    "kgf_propagate_vjp: NULL argument");
        KGF_REQUIRE(model->L == sector->L, KGF_EINVAL, "kgf_propagate_vjp: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(opts->direction == -1 || opts->direction == 1, KGF_EINVAL,
                    "kgf_propagate_vjp: direction must be -1 or +1");
        KGF_REQUIRE(nsteps >= 0 && quad_nodes >= 1 && quad_nodes <= 31, KGF_EINVAL,
                    "kgf_propagate_vjp: bad nsteps / quad_nodes");
        KGF_HIP(hipSetDevice(ctx->device));
        const int nth = n_theta(model);
        double* g = static_cast<double*>(workspace(ctx, "abi_grad", sizeof(double) * nth));
        KGF_HIP(hipMemsetAsync(g, 0, sizeof(double) * nth, ctx->stream));
        SilOpts o = to_sil_opts(opts);
        chain_adjoint(ctx, const_cast<kgf_model*>(model), sector, 1, reinterpret_cast<const double2*>(psi0),
                      sector->dim(), nsteps, o.dt, o.direction, o, quad_nodes, reinterpret_cast<double2*>(lam),
                      sector->dim(), g, 0);
        KGF_HIP(hipMemcpyAsync(host_grad, g, sizeof(double) * nth, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        ctx->ws.erase("adj_chain");
    });
}

int kgf_greens_neq_vjp(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                       const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb, int nt,
                       int steps_per_grid, const kgf_prop_opts* opts, const kgf_c128* host_W_lesser,
                       const kgf_c128* host_W_greater, int quad_nodes, double cg_tol, double* host_grad_ini,
                       double* host_grad, kgf_c128* host_G_lesser, kgf_c128* host_G_greater, double* host_E0,
                       int* host_cg_iters) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && H_ini && H && sector && gs_opts && v0 && host_orbs && host_E0, KGF_EINVAL,
                    "kgf_greens_neq_vjp: NULL argument");
        KGF_REQUIRE(H_ini->L == sector->L && H->L == sector->L, KGF_EINVAL,
                    "kgf_greens_neq_vjp: models and sector differ in L");
        check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && quad_nodes >= 1 && quad_nodes <= 31 &&
                        std::isfinite(cg_tol) && cg_tol > 0.0,
                    KGF_EINVAL, "kgf_greens_neq_vjp: bad sizes");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens_neq_vjp: bad ground-state options");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sector->L, KGF_EINVAL,
                        "kgf_greens_neq_vjp: orbital out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        VjpArgs A;
        A.sec = sector;
        A.orbs = host_orbs;
        A.norb = n_orb;
        A.nt = nt;
        A.spg = steps_per_grid;
        A.o = to_sil_opts(opts);
        A.nq = quad_nodes;
        A.cg_tol = cg_tol;
        A.cg_maxit = ctx->cg_max_iter > 0 ? ctx->cg_max_iter : 20000;
        std::vector<VjpMember> M(1);
        M[0].Hi = const_cast<kgf_model*>(H_ini);
        M[0].Hf = const_cast<kgf_model*>(H);
        M[0].v0 = reinterpret_cast<const double2*>(v0);
        M[0].Wl = reinterpret_cast<const double2*>(host_W_lesser);
        M[0].Wg = reinterpret_cast<const double2*>(host_W_greater);
        M[0].grad_ini = host_grad_ini;
        M[0].grad = host_grad;
        M[0].Gl = reinterpret_cast<double2*>(host_G_lesser);
        M[0].Gg = reinterpret_cast<double2*>(host_G_greater);
        M[0].E0 = host_E0;
        M[0].cg_iters = host_cg_iters;
        four_step_vjp(ctx, A, gs_opts, M);
        KGF_REQUIRE(!M[0].cg_failed, KGF_ENOCONV,
                    "kgf_greens_neq_vjp: the projected CG of the ground-state term stopped above cg_tol "
                    "(iteration limit or non-positive curvature); host_grad_ini is not reliable");
    });
}

int kgf_greens_neq_vjp_multi(kgf_ctx* ctx, int n_inst, const kgf_model* const* H_ini, const kgf_model* const* H,
                             const kgf_sector* const* sectors, const kgf_gs_opts* gs_opts, const kgf_c128* const* v0,
                             const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                             const kgf_prop_opts* opts, const kgf_c128* const* host_W_lesser,
                             const kgf_c128* const* host_W_greater, int quad_nodes, double cg_tol,
                             double* const* host_grad_ini, double* const* host_grad, double* host_E0,
                             int* host_cg_iters) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && n_inst >= 1 && H_ini && H && sectors && gs_opts && v0 && host_orbs && host_E0, KGF_EINVAL,
                    "kgf_greens_neq_vjp_multi: NULL argument");
        check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && quad_nodes >= 1 && quad_nodes <= 31 &&
                        std::isfinite(cg_tol) && cg_tol > 0.0,
                    KGF_EINVAL, "kgf_greens_neq_vjp_multi: bad sizes");
        KGF_REQUIRE(gs_opts->max_iter >= 1 && gs_opts->max_iter <= 4000 && gs_opts->check_every >= 1 &&
                        gs_opts->reorth >= 0 && gs_opts->reorth <= 2 && std::isfinite(gs_opts->tol) &&
                        gs_unique_opts_ok(gs_opts),
                    KGF_EINVAL, "kgf_greens_neq_vjp_multi: bad ground-state options");
        for (int i = 0; i < n_inst; ++i) {
            KGF_REQUIRE(H_ini[i] && H[i] && sectors[i] && v0[i], KGF_EINVAL, "kgf_greens_neq_vjp_multi: NULL instance");
            KGF_REQUIRE(H_ini[i]->L == sectors[i]->L && H[i]->L == sectors[i]->L && sectors[i]->dim() > 0, KGF_EINVAL,
                        "kgf_greens_neq_vjp_multi: model / sector mismatch or empty sector");
            for (int a = 0; a < n_orb; ++a)
                KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < sectors[i]->L, KGF_EINVAL,
                            "kgf_greens_neq_vjp_multi: orbital out of range");
        }
        KGF_HIP(hipSetDevice(ctx->device));
        std::vector<int> done(n_inst, 0);
        bool cg_failed = false;
        for (int i0 = 0; i0 < n_inst; ++i0) {
            if (done[i0]) continue;
            std::vector<VjpMember> M;
            for (int i = i0; i < n_inst; ++i) {
                const kgf_sector* a = sectors[i];
                const kgf_sector* b = sectors[i0];
                if (done[i] || a->L != b->L || a->n_up != b->n_up || a->n_dn != b->n_dn || !same_topology(H[i], H[i0]))
                    continue;
                done[i] = 1;
                VjpMember mb;
                mb.Hi = const_cast<kgf_model*>(H_ini[i]);
                mb.Hf = const_cast<kgf_model*>(H[i]);
                mb.v0 = reinterpret_cast<const double2*>(v0[i]);
                mb.Wl = host_W_lesser ? reinterpret_cast<const double2*>(host_W_lesser[i]) : nullptr;
                mb.Wg = host_W_greater ? reinterpret_cast<const double2*>(host_W_greater[i]) : nullptr;
                mb.grad_ini = host_grad_ini ? host_grad_ini[i] : nullptr;
                mb.grad = host_grad ? host_grad[i] : nullptr;
                mb.E0 = host_E0 + i;
                mb.cg_iters = host_cg_iters ? host_cg_iters + i : nullptr;
                M.push_back(mb);
            }
            VjpArgs A;
            A.sec = sectors[i0];
            A.orbs = host_orbs;
            A.norb = n_orb;
            A.nt = nt;
            A.spg = steps_per_grid;
            A.o = to_sil_opts(opts);
            A.nq = quad_nodes;
            A.cg_tol = cg_tol;
            A.cg_maxit = ctx->cg_max_iter > 0 ? ctx->cg_max_iter : 20000;
            four_step_vjp(ctx, A, gs_opts, M);
            for (const VjpMember& mb : M) cg_failed = cg_failed || mb.cg_failed;
        }
        KGF_REQUIRE(!cg_failed, KGF_ENOCONV,
                    "kgf_greens_neq_vjp_multi: the projected CG of a ground-state term stopped above cg_tol "
                    "(iteration limit or non-positive curvature); that instance's host_grad_ini is not reliable");
    });
}

}  // extern "C"
