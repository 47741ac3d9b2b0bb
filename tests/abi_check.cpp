// Host-side exercise of the C ABI for the sanitizer build: every call a
// client makes (context, model, sector, H.v, ground state, propagation with
// its error estimate, the four-step G in one call and step by step, the
// allocation-free propagation), the documented error returns, and the
// release of every handle.  Built with host AddressSanitizer and
// UndefinedBehaviorSanitizer (device code is not instrumented); the test
// that runs it checks its printed numbers against the oracle.
//
// Workload: the half-filled 8-site ring, t = 1, U = 4, sector (4, 4),
// D = 4,900; the quench adds a field 0.3 on site 0 to the initial
// Hamiltonian.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kgf.h"

#define HIP_OK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::printf("FAIL hip %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 2;                                                               \
        }                                                                           \
    } while (0)
#define KGF_OK_(x)                                                                        \
    do {                                                                                  \
        int r_ = (x);                                                                     \
        if (r_ != KGF_OK) {                                                               \
            std::printf("FAIL kgf %d (%s) at line %d\n", r_, kgf_last_error(), __LINE__); \
            return 3;                                                                     \
        }                                                                                 \
    } while (0)
#define EXPECT(c)                                                  \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL expectation at line %d\n", __LINE__); \
            return 4;                                              \
        }                                                          \
    } while (0)

int main() {
    const int L = 8;
    std::vector<int32_t> bi(L), bj(L);
    std::vector<double> t(L, 1.0), eps(L, 0.0), eps_f(L, 0.0), U(L, 4.0);
    for (int i = 0; i < L; ++i) {
        bi[i] = i;
        bj[i] = (i + 1) % L;
    }
    eps_f[0] = 0.3;
    EXPECT(kgf_version() == KGF_ABI_VERSION);

    kgf_ctx* ctx = nullptr;
    KGF_OK_(kgf_create(&ctx, 0, nullptr));
    kgf_model_desc d{L, L, bi.data(), bj.data(), t.data(), eps.data(), eps.data(), U.data()};
    kgf_model_desc di{L, L, bi.data(), bj.data(), t.data(), eps_f.data(), eps_f.data(), U.data()};
    kgf_model *H = nullptr, *Hi = nullptr;
    KGF_OK_(kgf_model_create(ctx, &d, &H));
    KGF_OK_(kgf_model_create(ctx, &di, &Hi));
    kgf_sector* sec = nullptr;
    KGF_OK_(kgf_sector_create(ctx, L, 4, 4, &sec));
    int64_t du = 0, dd = 0;
    KGF_OK_(kgf_sector_dims(sec, &du, &dd));
    const int64_t D = du * dd;
    EXPECT(D == 4900);

    // documented error returns (nothing is launched for them)
    kgf_sector* bad = nullptr;
    const int rs = kgf_sector_create(ctx, L, 9, 4, &bad);
    EXPECT((rs == KGF_EINVAL || rs == KGF_EUNSUPPORTED) && bad == nullptr);
    EXPECT(std::strlen(kgf_last_error()) > 0);
    std::vector<int32_t> many(200, 0), many_j(200, 1);
    std::vector<double> many_t(200, 1.0);
    kgf_model_desc dbad{L, 200, many.data(), many_j.data(), many_t.data(), eps.data(), eps.data(), U.data()};
    kgf_model* mbad = nullptr;
    EXPECT(kgf_model_create(ctx, &dbad, &mbad) != KGF_OK && mbad == nullptr);

    // start vector: deterministic, real, with overlap on every state
    std::vector<kgf_c128> hv(D);
    for (int64_t i = 0; i < D; ++i) hv[i] = {std::cos(0.37 * (double)i) + 0.1, 0.0};
    kgf_c128 *v0 = nullptr, *psi0 = nullptr, *work = nullptr, *w2 = nullptr;
    HIP_OK(hipMalloc(&v0, sizeof(kgf_c128) * D));
    HIP_OK(hipMalloc(&psi0, sizeof(kgf_c128) * D));
    HIP_OK(hipMalloc(&work, sizeof(kgf_c128) * 2 * D));
    HIP_OK(hipMalloc(&w2, sizeof(kgf_c128) * 2 * D));
    HIP_OK(hipMemcpy(v0, hv.data(), sizeof(kgf_c128) * D, hipMemcpyHostToDevice));

    kgf_gs_opts go{1e-12, 300, 1, 2, 1, 0.0, 8};
    kgf_gs_info gi{};
    double E0 = 0.0;
    KGF_OK_(kgf_ground_state(ctx, H, sec, &go, v0, psi0, &E0, &gi));
    EXPECT(gi.converged == 1 && gi.fidelity2 > 1.0 - 1e-10);

    // <0|H|0> = E0
    KGF_OK_(kgf_apply_h(ctx, H, sec, psi0, work, 1, D));
    std::vector<kgf_c128> p(D), hp(D);
    HIP_OK(hipMemcpy(p.data(), psi0, sizeof(kgf_c128) * D, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hp.data(), work, sizeof(kgf_c128) * D, hipMemcpyDeviceToHost));
    double eh = 0.0;
    for (int64_t i = 0; i < D; ++i) eh += p[i].re * hp[i].re + p[i].im * hp[i].im;

    // propagation of |0> and of a second column: |0> only changes phase
    HIP_OK(hipMemcpy(work, psi0, sizeof(kgf_c128) * D, hipMemcpyDeviceToDevice));
    HIP_OK(hipMemcpy(work + D, v0, sizeof(kgf_c128) * D, hipMemcpyDeviceToDevice));
    HIP_OK(hipMemcpy(w2, work, sizeof(kgf_c128) * 2 * D, hipMemcpyDeviceToDevice));
    kgf_prop_opts po{15, 0, 0.05, -1, 0.0, 1e-13};
    KGF_OK_(kgf_propagate(ctx, H, sec, work, 2, D, 10, &po, nullptr, nullptr));
    std::vector<kgf_c128> q(2 * D);
    HIP_OK(hipMemcpy(q.data(), work, sizeof(kgf_c128) * 2 * D, hipMemcpyDeviceToHost));
    double ov_re = 0.0, ov_im = 0.0;
    for (int64_t i = 0; i < D; ++i) {
        ov_re += p[i].re * q[i].re + p[i].im * q[i].im;
        ov_im += p[i].re * q[i].im - p[i].im * q[i].re;
    }
    kgf_prop_opts bad_po = po;
    bad_po.krylov_dim = 0;   // outside 1..128
    EXPECT(kgf_propagate(ctx, H, sec, work, 2, D, 1, &bad_po, nullptr, nullptr) == KGF_EUNSUPPORTED);
    bad_po = po;
    bad_po.dt = std::nan("");
    EXPECT(kgf_propagate(ctx, H, sec, work, 2, D, 1, &bad_po, nullptr, nullptr) == KGF_EINVAL);
    EXPECT(kgf_propagate(ctx, H, sec, work, 2, D, 1, nullptr, nullptr, nullptr) == KGF_EINVAL);

    // allocation-free propagation: bitwise the same states
    KGF_OK_(kgf_propagate_noalloc(ctx, H, sec, w2, 2, D, 10, &po, nullptr));
    std::vector<kgf_c128> q2(2 * D);
    HIP_OK(hipMemcpy(q2.data(), w2, sizeof(kgf_c128) * 2 * D, hipMemcpyDeviceToHost));
    EXPECT(std::memcmp(q.data(), q2.data(), sizeof(kgf_c128) * 2 * D) == 0);

    // the same steps with the a-posteriori error estimate
    HIP_OK(hipMemcpy(w2, psi0, sizeof(kgf_c128) * D, hipMemcpyDeviceToDevice));
    HIP_OK(hipMemcpy(w2 + D, v0, sizeof(kgf_c128) * D, hipMemcpyDeviceToDevice));
    double err = -1.0;
    KGF_OK_(kgf_propagate(ctx, H, sec, w2, 2, D, 10, &po, &err, nullptr));
    EXPECT(err >= 0.0 && err < 1e-6);

    // four-step G after the quench: one call, then step by step
    const int nt = 4, spg = 2, norb = 2;
    const int32_t orbs[norb] = {0, 1};   // site 0, spin up and spin down
    kgf_gs_opts g4{1e-12, 300, 1, 2, 0, 0.0, 8};
    kgf_prop_opts p4{15, 0, 0.05, -1, 0.0, 1e-13};
    const size_t ng = (size_t)nt * nt * norb * norb;
    std::vector<kgf_c128> Gl(ng), Gg(ng), Gl2(ng), Gg2(ng);
    double E0i = 0.0, E0r = 0.0;
    KGF_OK_(kgf_greens_neq(ctx, Hi, H, sec, &g4, v0, orbs, norb, nt, spg, &p4, 1, 3, 0, 0, 0.0, Gl.data(),
                           Gg.data(), nullptr, nullptr, nullptr, &E0i, nullptr));
    kgf_neq_run* run = nullptr;
    KGF_OK_(kgf_neq_run_create(ctx, Hi, H, sec, &g4, v0, orbs, norb, nt, spg, &p4, 3, &run, &E0r));
    EXPECT(kgf_neq_run_result(run, Gl2.data(), Gg2.data()) == KGF_EINVAL);   // intervals left
    kgf_neq_run_info ri{};
    int guard = 0;
    do {
        KGF_OK_(kgf_neq_run_advance(run, 1, &ri));
    } while (!ri.done && ++guard < 1000);
    EXPECT(ri.done == 1);
    KGF_OK_(kgf_neq_run_result(run, Gl2.data(), Gg2.data()));
    kgf_neq_run_destroy(run);
    EXPECT(E0r == E0i);
    EXPECT(std::memcmp(Gl.data(), Gl2.data(), sizeof(kgf_c128) * ng) == 0);
    EXPECT(std::memcmp(Gg.data(), Gg2.data(), sizeof(kgf_c128) * ng) == 0);

    // checkpoint between chunks, resume in a new run: the same G bitwise
    KGF_OK_(kgf_neq_run_create(ctx, Hi, H, sec, &g4, v0, orbs, norb, nt, spg, &p4, 3, &run, &E0r));
    int moved = 0;
    do {
        KGF_OK_(kgf_neq_run_advance(run, 1, &ri));
        ++moved;
    } while (!(ri.chunk_start && moved >= 5) && ++guard < 2000);
    size_t nimg = 0;
    KGF_OK_(kgf_neq_run_checkpoint(run, nullptr, 0, &nimg));
    std::vector<char> img(nimg);
    EXPECT(kgf_neq_run_checkpoint(run, img.data(), nimg - 1, nullptr) == KGF_EINVAL);   // short buffer
    KGF_OK_(kgf_neq_run_checkpoint(run, img.data(), nimg, &nimg));
    kgf_neq_run_destroy(run);
    KGF_OK_(kgf_neq_run_create(ctx, Hi, H, sec, &g4, v0, orbs, norb, nt, spg, &p4, 3, &run, &E0r));
    EXPECT(kgf_neq_run_restore(run, img.data(), sizeof(int)) == KGF_EINVAL);            // truncated image
    KGF_OK_(kgf_neq_run_restore(run, img.data(), nimg));
    EXPECT(kgf_neq_run_restore(run, img.data(), nimg) == KGF_EINVAL);                   // not a new run
    do {
        KGF_OK_(kgf_neq_run_advance(run, 1, &ri));
    } while (!ri.done && ++guard < 3000);
    std::fill(Gl2.begin(), Gl2.end(), kgf_c128{0.0, 0.0});
    std::fill(Gg2.begin(), Gg2.end(), kgf_c128{0.0, 0.0});
    KGF_OK_(kgf_neq_run_result(run, Gl2.data(), Gg2.data()));
    kgf_neq_run_destroy(run);
    EXPECT(std::memcmp(Gl.data(), Gl2.data(), sizeof(kgf_c128) * ng) == 0);
    EXPECT(std::memcmp(Gg.data(), Gg2.data(), sizeof(kgf_c128) * ng) == 0);

    HIP_OK(hipFree(v0));
    HIP_OK(hipFree(psi0));
    HIP_OK(hipFree(work));
    HIP_OK(hipFree(w2));
    kgf_sector_destroy(sec);
    kgf_model_destroy(H);
    kgf_model_destroy(Hi);
    kgf_destroy(ctx);

    std::printf("{\"E0\": %.17g, \"iters\": %d, \"fidelity2\": %.17g, \"E0_from_Hv\": %.17g, "
                "\"overlap_re\": %.17g, \"overlap_im\": %.17g, \"err_est\": %.17g, \"E0_ini\": %.17g, "
                "\"G_lesser\": [",
                E0, gi.iters, gi.fidelity2, eh, ov_re, ov_im, err, E0i);
    for (size_t i = 0; i < ng; ++i) std::printf("%s[%.17g, %.17g]", i ? ", " : "", Gl[i].re, Gl[i].im);
    std::printf("], \"G_greater\": [");
    for (size_t i = 0; i < ng; ++i) std::printf("%s[%.17g, %.17g]", i ? ", " : "", Gg[i].re, Gg[i].im);
    std::printf("]}\n");
    return 0;
}
