// Equilibrium spectra (Sec. 2 and Sec. 3):
//   * the conventional Lanczos Green's function G^(L)(omega), Eq. (gapprox),
//     evaluated as the continued fraction of the n x n tridiagonal matrix
//     (the same n-pole function as the sum over its Ritz pairs);
//   * the time-dependent Lanczos G(t), Eqs. (psit), (psigreen), on a fine time
//     grid: inside each short-iterative-Lanczos step the states at
//     intermediate times are combinations of that step's Krylov basis
//     (Eq. (udelta) with Delta t replaced by the fine time), so only m overlaps
//     <i0|v_j> per step are needed;
//   * the damped Fourier transform G(omega) = int_0^T dt e^{i omega t - eta t}
//     G(t) (the inverse of Eq. (ft) with the Lorentzian damping of Sec. 3),
//     trapezoid rule, fixed-order sums.
#include <cmath>

#include "kgf_internal.h"

namespace kgf {

namespace {

// out_j = sign * norm2 / (z_j - a_0 - b_1^2 / (z_j - a_1 - b_2^2 / ...)),
// z_j = sz * (omega_j + i eta) + shift.  One thread per frequency.
__global__ void k_cfrac(const double* __restrict__ a, const double* __restrict__ b, int n, double norm2,
                        const double* __restrict__ omega, int nw, double eta, double shift, double sz, double sign,
                        double2* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nw) return;
    const double zr = sz * omega[j] + shift, zi = sz * eta;
    double tr = 0.0, ti = 0.0;   // tail t = b_k^2 / (z - a_k - tail), bottom up
    for (int k = n - 1; k >= 1; --k) {
        const double dr = zr - a[k] - tr, di = zi - ti;
        const double den = dr * dr + di * di;
        const double bb = b[k] * b[k];
        tr = bb * dr / den;
        ti = -bb * di / den;
    }
    const double dr = zr - a[0] - tr, di = zi - ti;
    const double den = dr * dr + di * di;
    out[j] = make_double2(sign * norm2 * dr / den, -sign * norm2 * di / den);
}

// G_out[q] = ph(t_q) * sum_j coef[q][j] ov[j], t_q = t0 + (q + 1) dtf,
// ph(t) = pf * exp(-i dir E0 t) with pf = -i (greater) or +i (lesser)
__global__ void k_fine_values(const double2* __restrict__ coef, int m, const double2* __restrict__ ov, int nq,
                              double t0, double dtf, double E0, int dir, double pf, double2* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < m; ++j) {
        const double2 c = coef[(int64_t)q * m + j], o = ov[j];
        re += c.x * o.x - c.y * o.y;
        im += c.x * o.y + c.y * o.x;
    }
    const double t = t0 + (q + 1) * dtf;
    double sn, cs;
    sincos(-dir * E0 * t, &sn, &cs);   // exp(-i dir E0 t)
    const double vr = re * cs - im * sn, vi = re * sn + im * cs;
    out[q] = make_double2(-pf * vi, pf * vr);   // pf * i * v
}

// out_j = sum_k w_k e^{(i omega_j - eta) t_k} G_k, t_k = k dt, trapezoid weights
__global__ void k_fourier(const double2* __restrict__ G, int nt, double dt, const double* __restrict__ omega,
                          double eta, double2* __restrict__ out) {
    __shared__ double sh[2][kThreads / 64];
    const int j = blockIdx.x;
    const double w = omega[j];
    double re = 0.0, im = 0.0;
    for (int k = threadIdx.x; k < nt; k += blockDim.x) {
        const double t = k * dt;
        const double wt = (k == 0 || k == nt - 1) ? 0.5 * dt : dt;
        double sn, cs;
        sincos(w * t, &sn, &cs);
        const double e = wt * exp(-eta * t);
        const double2 g = G[k];
        re += e * (cs * g.x - sn * g.y);
        im += e * (cs * g.y + sn * g.x);
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = re;
        sh[1][wv] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0, i = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            r += sh[0][q];
            i += sh[1][q];
        }
        out[j] = make_double2(r, i);
    }
}

std::unique_ptr<kgf_sector> target_sector(kgf_ctx* ctx, const kgf_sector* sec, int spin, int delta) {
    const int nu = sec->n_up + (spin == 0 ? delta : 0), nd = sec->n_dn + (spin == 1 ? delta : 0);
    if (nu < 0 || nu > sec->L || nd < 0 || nd > sec->L) return nullptr;
    std::unique_ptr<kgf_sector> s(new kgf_sector());
    s->ctx = ctx;
    s->L = sec->L;
    s->n_up = nu;
    s->n_dn = nd;
    s->d_up = binom_host(sec->L, nu);
    s->d_dn = binom_host(sec->L, nd);
    s->masks_up.reserve(sizeof(uint32_t) * s->d_up);
    s->masks_dn.reserve(sizeof(uint32_t) * s->d_dn);
    build_masks(ctx, sec->L, nu, s->masks_up.as<uint32_t>(), s->d_up);
    build_masks(ctx, sec->L, nd, s->masks_dn.as<uint32_t>(), s->d_dn);
    return s;
}

}  // namespace

}  // namespace kgf

using namespace kgf;

extern "C" {

int kgf_greens_omega(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector, const kgf_c128* psi0, double E0,
                     int orbital, int n_lanczos, int reorth, const double* host_omega, int nw, double eta,
                     kgf_c128* host_G_greater, kgf_c128* host_G_lesser, int* host_steps) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && model && sector && psi0 && host_omega, KGF_EINVAL, "kgf_greens_omega: NULL argument");
        KGF_REQUIRE(model->L == sector->L, KGF_EINVAL, "kgf_greens_omega: model and sector L differ");
        KGF_REQUIRE(orbital >= 0 && (orbital >> 1) < sector->L && n_lanczos >= 1 && n_lanczos <= 4000 && nw >= 0 &&
                        reorth >= 0 && reorth <= 2 && std::isfinite(eta) && eta > 0.0,
                    KGF_EINVAL, "kgf_greens_omega: bad arguments");
        KGF_HIP(hipSetDevice(ctx->device));
        const int spin = orbital & 1;
        kgf_model* M = const_cast<kgf_model*>(model);
        double* wdev = static_cast<double*>(workspace(ctx, "sp_omega", sizeof(double) * (nw > 0 ? nw : 1)));
        double2* gdev = static_cast<double2*>(workspace(ctx, "sp_out", sizeof(double2) * (nw > 0 ? nw : 1)));
        if (nw > 0) KGF_HIP(hipMemcpy(wdev, host_omega, sizeof(double) * nw, hipMemcpyHostToDevice));
        for (int greater = 1; greater >= 0; --greater) {
            kgf_c128* dst = greater ? host_G_greater : host_G_lesser;
            if (!dst) continue;
            auto tgt = target_sector(ctx, sector, spin, greater ? +1 : -1);
            if (!tgt || tgt->dim() == 0) {
                for (int j = 0; j < nw; ++j) reinterpret_cast<double2*>(dst)[j] = make_double2(0.0, 0.0);
                if (host_steps) host_steps[greater ? 0 : 1] = 0;
                continue;
            }
            const int64_t Dt = tgt->dim();
            double2* i0 = static_cast<double2*>(workspace(ctx, "sp_i0", sizeof(double2) * Dt));
            apply_c(ctx, sector, tgt.get(), orbital, greater, reinterpret_cast<const double2*>(psi0), i0, 1,
                    sector->dim(), Dt);
            std::vector<double> a(n_lanczos), b(n_lanczos);
            double n2 = 0.0;
            const int taken = lanczos_tridiag(ctx, M, tgt.get(), i0, n_lanczos, reorth, a.data(), b.data(), &n2);
            if (host_steps) host_steps[greater ? 0 : 1] = taken;
            double* ab = static_cast<double*>(workspace(ctx, "sp_ab", sizeof(double) * 2 * n_lanczos));
            KGF_HIP(hipMemcpy(ab, a.data(), sizeof(double) * n_lanczos, hipMemcpyHostToDevice));
            KGF_HIP(hipMemcpy(ab + n_lanczos, b.data(), sizeof(double) * n_lanczos, hipMemcpyHostToDevice));
            if (nw > 0 && taken > 0) {
                // particle part: z = omega + i eta + E0; hole part: -(z - E0 ... ) see the header
                hipLaunchKernelGGL(k_cfrac, dim3((nw + kThreads - 1) / kThreads), dim3(kThreads), 0, ctx->stream, ab,
                                   ab + n_lanczos, taken, n2, wdev, nw, eta, E0, greater ? 1.0 : -1.0,
                                   greater ? 1.0 : -1.0, gdev);
                check_launch("k_cfrac");
                KGF_HIP(hipMemcpyAsync(dst, gdev, sizeof(double2) * nw, hipMemcpyDeviceToHost, ctx->stream));
                sync(ctx);
            } else {
                for (int j = 0; j < nw; ++j) reinterpret_cast<double2*>(dst)[j] = make_double2(0.0, 0.0);
            }
        }
    });
}

int kgf_greens_eq_fine(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector, const kgf_c128* psi0, double E0,
                       int orbital, int dagger, int nsteps, int nfine, const kgf_prop_opts* opts, kgf_c128* host_G) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && model && sector && psi0 && host_G, KGF_EINVAL, "kgf_greens_eq_fine: NULL argument");
        KGF_REQUIRE(model->L == sector->L, KGF_EINVAL, "kgf_greens_eq_fine: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(orbital >= 0 && (orbital >> 1) < sector->L && (dagger == 0 || dagger == 1) && nsteps >= 0 &&
                        nfine >= 1 && (int64_t)nsteps * nfine < (1LL << 31),
                    KGF_EINVAL, "kgf_greens_eq_fine: bad arguments");
        KGF_HIP(hipSetDevice(ctx->device));
        kgf_model* M = const_cast<kgf_model*>(model);
        double2* out = reinterpret_cast<double2*>(host_G);
        const int64_t ntot = (int64_t)nsteps * nfine + 1;
        auto tgt = target_sector(ctx, sector, orbital & 1, dagger ? +1 : -1);
        if (!tgt || tgt->dim() == 0) {
            for (int64_t j = 0; j < ntot; ++j) out[j] = make_double2(0.0, 0.0);
            return;
        }
        const int64_t Dt = tgt->dim();
        SilOpts o = to_sil_opts(opts);
        o.direction = dagger ? -1 : +1;   // G^>: e^{-iHt}; G^<: e^{+iHt}
        const int m = o.m;
        const double pf = dagger ? -1.0 : 1.0;   // G^> = -i(...), G^< = +i(...)
        double2* i0 = static_cast<double2*>(workspace(ctx, "fine_i0", sizeof(double2) * Dt * 2));
        double2* psi = i0 + Dt;
        apply_c(ctx, sector, tgt.get(), orbital, dagger, reinterpret_cast<const double2*>(psi0), i0, 1, sector->dim(),
                Dt);
        KGF_HIP(hipMemcpyAsync(psi, i0, sizeof(double2) * Dt, hipMemcpyDeviceToDevice, ctx->stream));
        double2* ov = static_cast<double2*>(workspace(ctx, "fine_ov", sizeof(double2) * (m + 1)));
        double2* coef = static_cast<double2*>(workspace(ctx, "fine_coef", sizeof(double2) * (size_t)nfine * m));
        double2* vals = static_cast<double2*>(workspace(ctx, "fine_vals", sizeof(double2) * (size_t)nfine));
        // t = 0: <i0|i0>
        block_dots(ctx, i0, Dt, 1, i0, Dt, 1, Dt, ov);
        double2 g0;
        KGF_HIP(hipMemcpyAsync(&g0, ov, sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        out[0] = make_double2(-pf * g0.y, pf * g0.x);
        const double dtf = o.dt / nfine;
        std::vector<int> col(nfine, 0), dir(nfine, o.direction);
        std::vector<double> tt(nfine);
        for (int q = 0; q < nfine; ++q) tt[q] = (q + 1) * dtf;
        tt[nfine - 1] = o.dt;
        for (int k = 0; k < nsteps; ++k) {
            sil_build(ctx, M, tgt.get(), psi, 1, Dt, o);
            double2* X = static_cast<double2*>(ctx->ws["sil_X"]->p);
            block_dots(ctx, i0, Dt, 1, psi, Dt, 1, Dt, ov);
            if (m > 1) block_dots(ctx, i0, Dt, 1, X, Dt, m - 1, Dt, ov + 1);
            sil_coefs(ctx, m, nfine, col.data(), tt.data(), dir.data(), 0.0, coef, m);
            hipLaunchKernelGGL(k_fine_values, dim3((nfine + kThreads - 1) / kThreads), dim3(kThreads), 0, ctx->stream,
                               coef, m, ov, nfine, k * o.dt, dtf, E0, o.direction, pf, vals);
            check_launch("k_fine_values");
            // advance: psi <- the state at the end of the step (the last request)
            sil_combine_multi(ctx, tgt.get(), psi, Dt, 1, m, 0, coef + (size_t)(nfine - 1) * m, m, 1, psi, Dt);
            KGF_HIP(hipMemcpyAsync(out + 1 + (int64_t)k * nfine, vals, sizeof(double2) * nfine, hipMemcpyDeviceToHost,
                                   ctx->stream));
            if ((k + 1) % 64 == 0 || k + 1 == nsteps) progress(ctx, "eq_fine", k + 1, nsteps);
        }
        sync(ctx);
    });
}

int kgf_fourier(kgf_ctx* ctx, const kgf_c128* host_G, int nt, double dt, double eta, const double* host_omega, int nw,
                kgf_c128* host_out) {
    return abi_guard([&] {
        KGF_REQUIRE(ctx && (nt == 0 || host_G) && (nw == 0 || (host_omega && host_out)), KGF_EINVAL,
                    "kgf_fourier: NULL argument");
        KGF_REQUIRE(nt >= 0 && nw >= 0 && std::isfinite(dt) && dt > 0.0 && std::isfinite(eta) && eta >= 0.0,
                    KGF_EINVAL, "kgf_fourier: bad arguments");
        if (nw == 0) return;
        KGF_HIP(hipSetDevice(ctx->device));
        double2* g = static_cast<double2*>(workspace(ctx, "ft_g", sizeof(double2) * (nt > 0 ? nt : 1)));
        double* w = static_cast<double*>(workspace(ctx, "ft_w", sizeof(double) * nw));
        double2* o = static_cast<double2*>(workspace(ctx, "ft_o", sizeof(double2) * nw));
        if (nt > 0) KGF_HIP(hipMemcpy(g, host_G, sizeof(double2) * nt, hipMemcpyHostToDevice));
        KGF_HIP(hipMemcpy(w, host_omega, sizeof(double) * nw, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_fourier, dim3(nw), dim3(kThreads), 0, ctx->stream, g, nt, dt, w, eta, o);
        check_launch("k_fourier");
        KGF_HIP(hipMemcpyAsync(host_out, o, sizeof(double2) * nw, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    });
}

}  // extern "C"
