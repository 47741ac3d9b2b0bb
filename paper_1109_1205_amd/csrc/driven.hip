// Time-dependent (driven) Hamiltonians, the extension the paper's outlook
// proposes (Sec. 6): instead of Krylov steps much shorter than every time
// scale of H(t), a fourth-order commutator-free exponential integrator with
// two exponentials per step.  For H(t) = sum_j f_j(t) H_j and a step
// [t, t + h] with Gauss-Legendre nodes t_1,2 = t + (1/2 -+ sqrt(3)/6) h,
//     U(t + h, t) = exp(-i h B_2) exp(-i h B_1),
//     B_1 = a_2 H(t_1) + a_1 H(t_2),   B_2 = a_1 H(t_1) + a_2 H(t_2),
//     a_1,2 = 1/4 -+ sqrt(3)/6
// (B_1 acts first).  H is linear in its parameter vector theta = (t_b,
// eps_up, eps_dn, U), so B_s is the Hamiltonian of theta_s = sum_j g_sj
// theta_j and each exponential is one short-iterative-Lanczos step of the
// ordinary kernels on a work model whose parameters are replaced per stage.
#include <cmath>
#include <vector>

#include "kgf_internal.h"

namespace kgf {

void driven_stage(kgf_model* work, const DriveTable& drv, int n, int stage) {
    const double a1 = 0.25 - std::sqrt(3.0) / 6.0, a2 = 0.25 + std::sqrt(3.0) / 6.0;
    const int nb = work->nb, L = work->L, nth = n_theta(work);
    const double* f1 = drv.f + (int64_t)n * 2 * drv.n_terms;   // f_j(t_1)
    const double* f2 = f1 + drv.n_terms;                       // f_j(t_2)
    std::vector<double> th(nth, 0.0);
    for (int j = 0; j < drv.n_terms; ++j) {
        const double g = stage == 0 ? a2 * f1[j] + a1 * f2[j] : a1 * f1[j] + a2 * f2[j];
        const double* tj = drv.theta + (int64_t)j * nth;
        for (int q = 0; q < nth; ++q) th[q] += g * tj[q];
    }
    model_set_params(work, th.data(), th.data() + nb, th.data() + nb + L, th.data() + nb + 2 * L);
}

}  // namespace kgf

using namespace kgf;

int kgf_propagate_driven(kgf_ctx* ctx, kgf_model* work, const kgf_sector* s, kgf_c128* psi, int nvec, int64_t ld,
                         int nsteps, int n_terms, const double* host_theta, const double* host_f,
                         const kgf_prop_opts* opts) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && work && s && opts, KGF_EINVAL, "kgf_propagate_driven: NULL handle");
        KGF_REQUIRE(work->L == s->L, KGF_EINVAL, "kgf_propagate_driven: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(opts->direction == -1, KGF_EINVAL, "kgf_propagate_driven: direction must be -1 (forward)");
        KGF_REQUIRE(nvec >= 0 && nsteps >= 0 && ld >= s->dim() && n_terms >= 1, KGF_EINVAL,
                    "kgf_propagate_driven: bad nvec / nsteps / ld / n_terms");
        if (nvec == 0 || nsteps == 0 || s->dim() == 0) return;
        KGF_REQUIRE(psi && host_theta && host_f, KGF_EINVAL, "kgf_propagate_driven: NULL array");
        const int nth = n_theta(work);
        for (int64_t i = 0; i < (int64_t)n_terms * nth; ++i)
            KGF_REQUIRE(std::isfinite(host_theta[i]), KGF_EINVAL, "kgf_propagate_driven: non-finite theta");
        for (int64_t i = 0; i < (int64_t)nsteps * 2 * n_terms; ++i)
            KGF_REQUIRE(std::isfinite(host_f[i]), KGF_EINVAL, "kgf_propagate_driven: non-finite drive value");
        KGF_HIP(hipSetDevice(ctx->device));
        const SilOpts o = to_sil_opts(opts);
        const DriveTable drv{n_terms, host_theta, host_f};
        for (int n = 0; n < nsteps; ++n) {
            for (int stage = 0; stage < 2; ++stage) {
                driven_stage(work, drv, n, stage);
                sil_propagate(ctx, work, s, reinterpret_cast<double2*>(psi), nvec, ld, 1, o);
            }
            if ((n + 1) % 16 == 0 || n + 1 == nsteps) progress(ctx, "driven", n + 1, nsteps);
        }
    });
}
