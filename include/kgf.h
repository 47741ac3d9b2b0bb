/*
 * kgf.h -- C ABI of the Krylov-space Green's-function library (libkgf.so).
 *
 * Method: Balzer, Gdaniec & Potthoff, "Krylov-space approach to the
 * equilibrium and the nonequilibrium single-particle Green's function".
 * All arithmetic runs in hand-written HIP kernels for gfx950 in FP64
 * (complex128 state vectors).
 *
 * Conventions shared by every call
 * --------------------------------
 * Model (Sec. 3 Hubbard model, Sec. 4 Anderson model with the field of
 * Eq. (hfi), written with site-resolved parameters):
 *     H = - sum_b t_b sum_s (c+_{i_b s} c_{j_b s} + h.c.)
 *         + sum_{i s} eps_{i s} n_{i s} + sum_i U_i n_{i up} n_{i dn}
 * Basis of a sector (N_up, N_dn) (occupation-number basis, Sec. 2; N and
 * S_z conservation, Sec. 4): per spin the L-bit masks with N bits set in
 * ascending numeric order; a state vector is a D_up x D_dn row-major matrix
 * (element (u, d) at index u*D_dn + d).  Fermion order: all up modes
 * before all down modes, sites ascending, bit i = site i.
 * Orbital codes: alpha = 2*site + spin (spin 0 = up, 1 = down).
 *
 * Memory: pointers named host_* are host memory; every other pointer is
 * device memory on the context's device.  The caller owns all buffers it
 * passes; the library never frees them.  Buffers must stay valid until the
 * context's stream has been synchronised.  Handles returned by *_create
 * are owned by the caller and released with the matching *_destroy.
 * Calls that write host_* outputs synchronise the stream; the others are
 * asynchronous on the context's stream.
 *
 * Errors: every int-returning call returns KGF_OK (0) or a negative code;
 * kgf_last_error() then describes the failure (thread-local, valid until
 * the next call on the same thread).  No exception crosses the ABI.
 * Threading: one context per host thread.
 */
#ifndef KGF_H
#define KGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KGF_OK            0
#define KGF_EINVAL       -1   /* bad argument (size, pointer, range, NaN)   */
#define KGF_ENOMEM       -2   /* device allocation failed or would not fit */
#define KGF_EHIP         -3   /* HIP runtime error                          */
#define KGF_ENOCONV      -4   /* ground-state Lanczos did not converge      */
#define KGF_EUNSUPPORTED -5   /* size outside the supported range          */
#define KGF_EDEGENERATE  -6   /* two Lanczos starts reached different ground states */

/* complex128, interleaved (re, im); layout-compatible with torch.complex128 */
typedef struct { double re, im; } kgf_c128;

typedef struct kgf_ctx kgf_ctx;
typedef struct kgf_model kgf_model;
typedef struct kgf_sector kgf_sector;

/* ---- context ------------------------------------------------------------
 * kgf_create: bind a context to HIP device `hip_device` and the stream
 * `hip_stream` (a hipStream_t, borrowed, may be NULL for the null stream).
 * All kernels of calls on this context are launched on that stream. */
int  kgf_create(kgf_ctx** out, int hip_device, void* hip_stream);
/* kgf_destroy frees the context's workspaces.  Models and sectors created on
 * it must be destroyed first (their destroy synchronises on the context's
 * stream); handles still alive afterwards must not be passed to any call. */
void kgf_destroy(kgf_ctx* ctx);
int  kgf_set_stream(kgf_ctx* ctx, void* hip_stream);
const char* kgf_last_error(void);
/* ABI version of this header: incremented whenever a declaration, a struct
 * layout or the meaning of an argument changes.  kgf_version returns the
 * version the library was built with; a caller compiled against this header
 * compares it with KGF_ABI_VERSION before any other call. */
#define KGF_ABI_VERSION 2
int  kgf_version(void);

/* ---- model ----------------------------------------------------------------
 * Parameters of H (see the header comment).  Bonds are undirected; each
 * bond contributes both hopping directions (Sec. 3 sum over <ij>, Sec. 4
 * "+ H.c.").  All arrays are host memory and are copied.
 * Limits: 1 <= L <= 24, 0 <= n_bonds <= 127, 0 <= bond_i, bond_j < L,
 * bond_i != bond_j, all values finite (KGF_EINVAL / KGF_EUNSUPPORTED). */
typedef struct {
    int L;
    int n_bonds;
    const int32_t* bond_i;     /* host [n_bonds] */
    const int32_t* bond_j;     /* host [n_bonds] */
    const double*  t_bond;     /* host [n_bonds] hopping amplitudes t_b   */
    const double*  eps_up;     /* host [L] on-site energies, spin up      */
    const double*  eps_dn;     /* host [L] on-site energies, spin down    */
    const double*  U;          /* host [L] Hubbard interaction per site   */
} kgf_model_desc;

int  kgf_model_create(kgf_ctx* ctx, const kgf_model_desc* desc, kgf_model** out);
void kgf_model_destroy(kgf_model* model);
/* kgf_model_set_params: replace the parameters (t_bond, eps_up, eps_dn, U) of
 * a model in place; L and the bond list must equal the model's (KGF_EINVAL
 * otherwise).  Waits for the context's stream first, so work already issued
 * uses the old values; hopping tables built for the model are kept (they
 * depend on the bond topology only) and their on-site energies recomputed.
 * Instance sets built from the model (kgf_greens_neq_multi) must not run
 * concurrently with the change. */
int  kgf_model_set_params(kgf_model* model, const kgf_model_desc* desc);
/* kgf_model_get_params: copy the model's current parameters to host arrays
 * t [n_bonds], eps_up [L], eps_dn [L], U [L] (any may be NULL) -- after
 * kgf_propagate_driven / kgf_greens_neq_driven, the last stage's. */
int  kgf_model_get_params(const kgf_model* model, double* host_t, double* host_eps_up, double* host_eps_dn,
                          double* host_U);

/* ---- sector basis (Sec. 2 occupation-number basis; Sec. 4 N, S_z) --------
 * kgf_sector_create builds, on the device, the ascending mask tables of
 * the (n_up, n_dn) sector of an L-site cluster by unranking the
 * combinatorial number system (bit-exact integer work). */
int  kgf_sector_create(kgf_ctx* ctx, int L, int n_up, int n_dn, kgf_sector** out);
void kgf_sector_destroy(kgf_sector* sector);
int  kgf_sector_dims(const kgf_sector* sector, int64_t* d_up, int64_t* d_dn);
/* copy the mask table of one spin (0 up, 1 down) to host [D_spin] */
int  kgf_sector_states(kgf_ctx* ctx, const kgf_sector* sector, int spin, uint32_t* host_masks);
/* combinatorial rank of `n` masks (device uint32 in, device int64 out);
 * masks whose popcount differs from the sector's N_spin give -1. */
int  kgf_sector_rank(kgf_ctx* ctx, const kgf_sector* sector, int spin,
                     const uint32_t* masks, int64_t n, int64_t* ranks);

/* ---- hopping table (the single-species hopping matrix of H) ---------------
 * For the n-particle masks of an L-site model, row r lists the nonzeros of
 * <s_r| -sum_b t_b (c+_i c_j + c+_j c_i) |s'> as packed uint32 entries
 *     bits 0..23 column rank, bits 24..30 bond index, bit 31 sign
 * (value = -t_bond * (sign ? -1 : +1)); ELL layout entry[k*D + r] for
 * k < count[r] <= width.  Copies to host: count [D], entries [width*D],
 * *host_width = width.  Used to check the device-built table bit-exactly. */
int  kgf_hop_table(kgf_ctx* ctx, const kgf_model* model, int n,
                   int32_t* host_count, uint32_t* host_entries, int* host_width);

/* ---- H.v (Sec. 3 Hubbard H, Sec. 4 SIAM H) --------------------------------
 * w[c] = H v[c] for nvec vectors in the sector; vector c starts at
 * v + c*ld (ld >= D, in elements).  v and w must not overlap. */
int  kgf_apply_h(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                 const kgf_c128* v, kgf_c128* w, int nvec, int64_t ld);

/* ---- c_alpha / c+_alpha (Eqs. (psit), (glesser); Sec. 4 step (iii)) --------
 * w[c] = c_alpha v[c] (dagger = 0) or c+_alpha v[c] (dagger = 1); v in
 * `src`, w in `dst`, which must be the sector with one particle of the
 * orbital's spin less (more).  Fermion sign: (-1)^(occupied modes before
 * alpha).  w is fully written (zeros where the operator gives nothing). */
int  kgf_apply_c(kgf_ctx* ctx, const kgf_sector* src, const kgf_sector* dst,
                 int orbital, int dagger, const kgf_c128* v, kgf_c128* w,
                 int nvec, int64_t ld_src, int64_t ld_dst);

/* ---- ground state (Sec. 2; Sec. 4 step (i)) --------------------------------
 * Lanczos recursion (Eq. (recursion)) from the start vector v0 with
 * Gram-Schmidt reorthogonalisation (reorth: 1 classical GS, 2 twice), T_k
 * diagonalised on the device (Eq. (tdiag)); stops when the Ritz residual
 * b_{k+1}|y_k| <= tol * max(1, |E0|) (checked every check_every steps) or
 * at max_iter.  psi0 (device, D) receives the normalised Ritz vector
 * (Eq. (eigen)).  Returns KGF_ENOCONV (psi0, E0 still written) when not
 * converged.  Workspace: (max_iter + 1) vectors of D complex128.
 * Uniqueness (the method assumes a nondegenerate ground state, Sec. 2 and
 * Sec. 4 step (i)): with unique_check = 1 a second recursion runs from a
 * second start vector -- real entries uniform in [-1, 1) from the SplitMix64
 * generator (Steele, Lea, Flood 2014) at counter i for entry i, seeded with
 * unique_seed -- and fidelity2 = |<0_a|0_b>|^2 of the two normalised Ritz
 * vectors is reported; below 1 - unique_tol (0: 1e-10) the call returns
 * KGF_EDEGENERATE, with psi0 and E0 of the first start written.  The same
 * options apply to the ground state inside the four-step drivers.
 * unique_check = 0 (the default of a zeroed struct) skips the second run
 * (fidelity2 = -1). */
typedef struct {
    double   tol;
    int      max_iter;
    int      check_every;
    int      reorth;
    int      unique_check;
    double   unique_tol;
    uint64_t unique_seed;
} kgf_gs_opts;
typedef struct {
    int    iters;
    int    converged;
    double residual;
    double fidelity2;
} kgf_gs_info;
int  kgf_ground_state(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                      const kgf_gs_opts* opts, const kgf_c128* v0, kgf_c128* psi0,
                      double* host_E0, kgf_gs_info* host_info);

/* ---- short-iterative-Lanczos propagation (Sec. 3, Eqs. (newstate), (udelta))
 * Each of nvec vectors psi[c] (at psi + c*ld) is advanced nsteps times by
 *   direction -1: exp(-i H dt);  +1: exp(+i H dt);  0: exp(-(H - shift) dt)
 * using a Krylov space of dimension krylov_dim (<= 128) rebuilt at every
 * step (restart); exp(-+i T dt) e_1 by Taylor substeps, or by an implicit-QL
 * eigen-decomposition of T when ||T dt|| is large, in one block of one or two
 * wavefronts.  The
 * vectors of a batch run independent recursions (own a_k, b_k, T).
 * reorth: 0 none, 1 classical GS, 2 classical GS twice.  A recursion
 * stops early (exactly) when b_{k+1} <= breakdown_tol * max(|a_j|, b_j).
 * host_err_est (or NULL): the largest, over columns and steps, a-posteriori
 * estimate of one step's error in the 2-norm, the Krylov residual of the
 * approximation of Eq. (udelta) integrated over the step,
 *     beta0 * b_m * int_0^dt |[f_tau(T_m) e_1]_{m-1}| dtau   (16-point Gauss-Legendre),
 *     f_tau(T) = exp(-+i T tau) or exp(-(T - shift) tau)
 * (b_m: the norm the recursion would carry into a further step; zero after
 * a breakdown, where the step is exact).  For the real-time directions the
 * propagator is unitary and this bounds the step's error up to the
 * quadrature.  Asking for it costs the tridiagonal exponential at the 16
 * nodes, one more vector update per step, and synchronises the stream.
 * host_norm_drift (or NULL): the largest, over columns and steps, of
 * | ||psi after the step|| / ||psi before it|| - 1 |.  The real-time steps are
 * unitary (Sec. 3), so this measures the loss of orthogonality of the Krylov
 * basis and rounding; a value far above 1e-14 flags a step the caller should
 * rerun with reorthogonalisation or a smaller dt (for direction 0 the norm is
 * not conserved and the value is the decay itself).  Costs one norm pass per
 * step and synchronises the stream.
 * Workspace: krylov_dim * nvec vectors of D complex128. */
typedef struct {
    int    krylov_dim;
    int    reorth;
    double dt;
    int    direction;
    double shift;
    double breakdown_tol;
} kgf_prop_opts;
int  kgf_propagate(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                   kgf_c128* psi, int nvec, int64_t ld, int nsteps, const kgf_prop_opts* opts,
                   double* host_err_est, double* host_norm_drift);

/* ---- allocation-free propagation ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * kgf_propagate_noalloc does what kgf_propagate does, with the same kernels
 * and bitwise the same results, but takes every buffer it needs (Krylov
 * slots, per-column scalars, reduction partials) from a fixed device array
 * of KGF_NOALLOC_SCRATCH_BYTES per GPU, resolved at kgf_create and held until
 * the process ends; it calls no allocator.  Limits: the scratch must hold
 * krylov_dim * nvec * D complex128 plus small per-column arrays, else
 * KGF_EUNSUPPORTED (e.g. D = 63,504, krylov_dim 15: up to 4 columns); the
 * model's hopping tables for the sector's particle numbers must already
 * exist (one kgf_apply_h or kgf_propagate on the sector builds them), else
 * KGF_EINVAL.  All calls on one GPU share the array: calls that overlap in
 * time on that GPU (another thread, another stream) race; calls issued in
 * order on one stream do not.  Nothing in the array has to start at zero:
 * every value a step reads is written earlier in the same step. */
#define KGF_NOALLOC_SCRATCH_BYTES (64ull << 20)
int  kgf_propagate_noalloc(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                           kgf_c128* psi, int nvec, int64_t ld, int nsteps, const kgf_prop_opts* opts,
                           double* host_err_est);

/* ---- equilibrium Green's function (Sec. 3, Eqs. (psit), (psigreen), eta=0)
 *   G^>_{ij}(t_k) = -i e^{+i E0 t_k} <c+_i 0| e^{-iH t_k} |c+_j 0>
 *   G^<_{ij}(t_k) = +i e^{-i E0 t_k} <c_j 0| e^{+iH t_k} |c_i 0>
 * on t_k = k * steps_per_grid * opts->dt, k = 0..nt-1, for the n_orb
 * orbital codes in host_orbs.  psi0: ground state in `sector` (device).
 * batch: number of vectors propagated together (0 = all, 1 = one by one).
 * Outputs host [nt][n_orb][n_orb]; entries between orbitals of different
 * spin are zero. */
int  kgf_greens_eq(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                   const kgf_c128* psi0, double E0, const int32_t* host_orbs, int n_orb,
                   int nt, int steps_per_grid, const kgf_prop_opts* opts, int batch,
                   kgf_c128* host_G_greater, kgf_c128* host_G_lesser);

/* ---- driven Hamiltonians (Sec. 6, outlook) ---------------------------------
 * kgf_propagate_driven: psi[c] (at psi + c*ld, device, nvec columns) is
 * advanced nsteps steps of opts->dt under H(t) = sum_j f_j(t) H_j, where H_j
 * has the parameter vector host_theta[j*n_theta .. ] = (t_b, eps_up, eps_dn,
 * U) on the bond list of `work`, by the fourth-order commutator-free
 * exponential integrator with two exponentials per step:
 *   U(t+h, t) = exp(-i h B_2) exp(-i h B_1),
 *   B_1 = a_2 H(t_1) + a_1 H(t_2),  B_2 = a_1 H(t_1) + a_2 H(t_2),
 *   a_1,2 = 1/4 -+ sqrt(3)/6,  t_1,2 = t + (1/2 -+ sqrt(3)/6) h.
 * host_f[(n*2 + q)*n_terms + j] = f_j(t_q) of step n (the caller evaluates
 * its drive at the Gauss nodes).  Each exponential is one SIL step
 * (krylov_dim, reorth, breakdown_tol from opts; direction must be -1);
 * `work` (same L and bonds) has its parameters replaced per stage and holds
 * the last stage's on return. */
int  kgf_propagate_driven(kgf_ctx* ctx, kgf_model* work, const kgf_sector* sector, kgf_c128* psi, int nvec,
                          int64_t ld, int nsteps, int n_terms, const double* host_theta, const double* host_f,
                          const kgf_prop_opts* opts);

/* kgf_greens_neq_driven: the four-step G^<, G^> (Sec. 4) with the driven final
 * Hamiltonian of kgf_propagate_driven.  |0> = ground state of H_ini in `sector`
 * (from v0, gs_opts); Phi(t_k) = U(t_k, 0)|0> by the commutator-free
 * integrator with steps h = opts->dt from t = 0, t_k = k * steps_per_grid * h,
 * k = 0..nt-1; host_f holds the (nt-1)*steps_per_grid steps in the layout of
 * kgf_propagate_driven (step n starts at t = n h).  With U^+ the adjoint stage
 * exponentials in reverse order,
 *   G^<_ab(t, t') = +i <Psi_b(t')|Psi_a(t)>,  Psi_a(t) = U(t, 0)^+ c_a Phi(t),
 *   G^>_ab(t, t') = -i <chi_a(t)|chi_b(t')>,  chi_a(t) = U(t, 0)^+ c+_a Phi(t),
 * evaluated by one backward sweep per spin and per c / c+ that carries the
 * columns U(t_j, t_s)^+ c_a Phi(t_j) and dots them with c_b Phi(t_s) at every
 * mesh time t_s <= t_j (t_j < t_s from G_ab(t, t')* = -G_ba(t', t)).
 * batch: most columns in one sweep block (0 = as many as fit in memory).
 * Outputs host [nt][nt][n_orb][n_orb] (zero between orbitals of different
 * spin; either may be NULL) and E0.  `work` (not H_ini; same L and bonds as
 * the terms) is left holding the last stage's parameters.  KGF_ENOCONV if the
 * ground state does not converge. */
int  kgf_greens_neq_driven(kgf_ctx* ctx, const kgf_model* H_ini, kgf_model* work, const kgf_sector* sector,
                           const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                           int nt, int steps_per_grid, const kgf_prop_opts* opts, int batch, int n_terms,
                           const double* host_theta, const double* host_f, kgf_c128* host_G_lesser,
                           kgf_c128* host_G_greater, double* host_E0);

/* ---- four-time two-particle Green's functions (Sec. 6 outlook) --------------
 * kgf_greens2_neq: after the ground state |0> of H_ini in `sector` (from v0,
 * gs_opts) and the switch to H at t = 0, on the mesh t_k = k * steps_per_grid
 * * opts->dt, k < nt:
 *   host_chi[k1][k2][k3][k4][a][b][c][d]
 *     = <0| O1_a(t_k1) O2_b(t_k2) O3_c(t_k3) O4_d(t_k4) |0>,
 * O(t) = e^{iHt} O e^{-iHt}, O_m = c+ where bit (4 - m) of `pattern` is set,
 * else c (pattern 0b1100 = 12: c+ c+ c c; exactly two bits set, KGF_EINVAL
 * otherwise), for the n_orb orbital codes (site*2+spin) in host_orbs; zero
 * where the spins cannot match.  Evaluated as the scalar products of the
 * two-time states O2_b(t2)^+ O1_a(t1)^+ |0> and O3_c(t3) O4_d(t4) |0> (SIL
 * steps of opts; the inner operator's state carried through the mesh, the
 * outer operator applied at every mesh time, all states returned to t = 0 in
 * one sweep).  host_chi (caller-owned, nt^4 n_orb^4 complex128, at most 2^28
 * entries) and host_E0 are host arrays.  KGF_ENOCONV if the ground state does
 * not converge. */
int  kgf_greens2_neq(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                     const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                     int nt, int steps_per_grid, const kgf_prop_opts* opts, int pattern, kgf_c128* host_chi,
                     double* host_E0);

/* ---- nonequilibrium cluster-perturbation theory (Sec. 5, Eq. (cpteq)) -------
 * Contour: the Keldysh contour on the mesh t_k = k dt, k < nt (forward, then
 * backward); a contour function is G^> where its first time is later on the
 * contour, G^< where earlier; contour integrals by the trapezoid rule on each
 * branch with the integrand's jumps at nodes (mean of the one-sided limits at
 * interior nodes, the limit from inside the branch at branch ends).  The initial state is the
 * ground state of the disconnected system (cluster and bath), the
 * inter-cluster hopping acts for t > 0.
 *
 * kgf_bath_chain: Eqs. (gb1), (gb2) for the first site of an L_b-site chain
 * with hopping -T_b between neighbours and inverse temperature beta (INFINITY:
 * the ground state; levels at zero half filled), written to the device meshes
 * G_lesser, G_greater [nt][nt] (complex128, caller-owned).
 *
 * kgf_necpt: the cluster block of G = (G'^-1 - V)^-1 for a cluster linked at
 * its site `boundary` by the hopping V to bath site 1: with the bath
 * eliminated, G = G^c + G^c * Sigma * G, Sigma = V^2 G^b_11 on `boundary`.
 * Inputs (device, complex128): the cluster's Gc_lesser, Gc_greater
 * [nt][nt][n_c][n_c] (one spin; e.g. kgf_greens_neq) and the bath's
 * Gb_lesser, Gb_greater [nt][nt]; outputs G_lesser, G_greater
 * [nt][nt][n_c][n_c] (device, caller-owned, not aliasing the inputs).
 * Workspace ~16 (2 nt n_c)^2 bytes.  KGF_EUNSUPPORTED if 2 nt n_c > 65536,
 * KGF_EINVAL for a singular contour matrix.  The error of the scheme is
 * second order in dt. */
int  kgf_bath_chain(kgf_ctx* ctx, int L_b, double T_b, double beta, int nt, double dt,
                    kgf_c128* G_lesser, kgf_c128* G_greater);
int  kgf_necpt(kgf_ctx* ctx, int nt, int n_c, int boundary, double dt, double V,
               const kgf_c128* Gc_lesser, const kgf_c128* Gc_greater, const kgf_c128* Gb_lesser,
               const kgf_c128* Gb_greater, kgf_c128* G_lesser, kgf_c128* G_greater);

/* ---- NE-CPT on the Keldysh-Matsubara contour (Sec. 5, Eq. (cpteq)) ----------
 * The contour 0 -> t_max -> 0 -> -i beta: nt real mesh points t_k = k dt on
 * each real branch, then ntau >= 2 points z = -i tau_j, tau_j = j dtau,
 * (ntau-1) dtau = beta, later than both real branches.  The hopping V acts on
 * every branch, so the connected system's initial state is its equilibrium
 * state at beta, built by the CPT equation itself (Sec. 5 treats the initial
 * state by CPT through a Matsubara branch).  The imaginary branch enters the
 * contour integral with the weight -i dtau (trapezoid, halved at its ends)
 * and the equal-point rules of kgf_necpt; second order in dt and dtau.
 * A contour function is passed by its components (device, complex128, over
 * the orbitals [..][n][n]; n = n_c for the cluster, 1 for the bath's site 1):
 *   lesser, greater [nt][nt] = G^<, G^>(t_a, t_b);
 *   mixed [nt][ntau] = G^<(t_a, -i tau_j) (kgf_greens_neq's G_mixed);
 *   mixed_left [ntau][nt] = G^>(-i tau_j, t_b) (G_mixed_left);
 *   vert_greater [ntau] = G^>(-i tau_d, -i 0) = i G^M(+tau_d);
 *   vert_lesser [ntau] = G^<(-i 0, -i tau_d) = i G^M(-tau_d).
 * The members are read only by kgf_necpt_contour.
 * kgf_bath_chain_contour: Eqs. (gb1), (gb2) on complex contour times for
 * site 1 of an L_b-site chain (hopping -T_b, no quench) at inverse
 * temperature beta (INFINITY: the ground state), written to every member of
 * *out (n = 1; caller-owned device memory).
 * kgf_necpt_contour: the cluster block of G = (G'^-1 - V)^-1 for a cluster
 * linked at site `boundary` by V to bath site 1 (bath eliminated: Sigma =
 * V^2 G^b_11 on `boundary`).  Outputs (device, caller-owned): G_lesser,
 * G_greater [nt][nt][n_c][n_c]; G_mixed [nt][ntau][n_c][n_c] and
 * G_mixed_left [ntau][nt][n_c][n_c] or NULL.  Workspace
 * ~16 ((2 nt + ntau) n_c)^2 bytes.  KGF_EUNSUPPORTED if (2 nt + ntau) n_c >
 * 65536, KGF_EINVAL for a singular contour matrix or an incomplete function. */
typedef struct {
    kgf_c128* lesser;
    kgf_c128* greater;
    kgf_c128* mixed;
    kgf_c128* mixed_left;
    kgf_c128* vert_greater;
    kgf_c128* vert_lesser;
} kgf_contour_fn;
int  kgf_bath_chain_contour(kgf_ctx* ctx, int L_b, double T_b, double beta, int nt, double dt, int ntau,
                            double dtau, const kgf_contour_fn* out);
/* kgf_cluster_contour: a cluster's contour function (the members of *out,
 * device, caller-owned, shapes as above with n = n_c) from the host outputs
 * of kgf_greens_neq with ntau >= 2 (G_lesser, G_greater [nt][nt][n_orb][n_orb],
 * G_matsubara [2][ntau][..], G_mixed [nt][ntau][..], G_mixed_left [ntau][nt][..]),
 * for the orbitals host_sel[0..n_c) (NULL: all, n_c = n_orb): lesser, greater,
 * mixed, mixed_left as given, vert_greater = i G^M(+tau), vert_lesser =
 * i G^M(-tau) (Sec. 4 mixed and Matsubara functions, Sec. 5 Eq. (cpteq)).
 * kms = 1 completes these ground-state functions for an imaginary branch of
 * finite length beta = (ntau - 1) dtau: in an equilibrium at beta dominated
 * by the ground state, the states of N -+ 1 particles reached by c, c+ enter
 * near the far end of the branch, where they are the same ground-state
 * products read at beta - tau:
 *   vert_greater(tau) = i G^M(+tau) - i G^M(-(beta - tau)),
 *   vert_lesser(tau)  = i G^M(-tau) - i G^M(+(beta - tau)),
 *   mixed_ab(t, tau)  = G^|_ab(t, tau) + conj(G^|_ba(beta - tau, t)),
 *   mixed_left_ab(tau, t) = G^|_ab(tau, t) + conj(G^|_ba(t, beta - tau))
 * (G(-i beta, z') = -G(0, z') then holds up to terms of order e^{-beta Delta},
 * Delta the cluster's lowest excitation energy in the sectors involved);
 * kms = 0 leaves them as the ground state gives them.  Synchronises before
 * returning (the host arrays are read on the stream).  KGF_EINVAL for a NULL
 * member, an orbital index outside [0, n_orb) or kms not 0 / 1. */
int  kgf_cluster_contour(kgf_ctx* ctx, int nt, int ntau, int n_orb, const kgf_c128* host_G_lesser,
                         const kgf_c128* host_G_greater, const kgf_c128* host_G_matsubara,
                         const kgf_c128* host_G_mixed, const kgf_c128* host_G_mixed_left, const int* host_sel,
                         int n_c, int kms, const kgf_contour_fn* out);
int  kgf_necpt_contour(kgf_ctx* ctx, int nt, int ntau, int n_c, int boundary, double dt, double dtau, double V,
                       const kgf_contour_fn* Gc, const kgf_contour_fn* Gb, kgf_c128* G_lesser,
                       kgf_c128* G_greater, kgf_c128* G_mixed, kgf_c128* G_mixed_left);

/* ---- equilibrium spectra (Sec. 2, Sec. 3) ----------------------------------
 * kgf_greens_omega: the conventional Lanczos Green's function of Eq. (gapprox)
 * for orbital a (site*2+spin) from the ground state psi0 (device, in `sector`)
 * with energy E0, at the n_lanczos-step tridiagonal matrix (reorth 0..2 passes
 * of Gram-Schmidt), evaluated as the continued fraction on host_omega[nw]:
 *   host_G_greater[j] = <i0|(omega_j + i eta + E0 - H)^-1|i0>,  i0 = c+_a |0>,
 *   host_G_lesser[j]  = <i0|(omega_j + i eta - E0 + H)^-1|i0>,  i0 = c_a |0>;
 * the retarded G_aa(omega) is their sum and A = -Im G / pi.  eta > 0.
 * host_steps[0..1] (or NULL) receive the Lanczos steps taken (fewer than
 * n_lanczos when the Krylov space is exhausted).  Either output may be NULL. */
int  kgf_greens_omega(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                      const kgf_c128* psi0, double E0, int orbital, int n_lanczos, int reorth,
                      const double* host_omega, int nw, double eta, kgf_c128* host_G_greater,
                      kgf_c128* host_G_lesser, int* host_steps);

/* kgf_greens_eq_fine: the time-dependent Lanczos G of Eqs. (psit), (psigreen)
 * for orbital a on a fine grid: nsteps short-iterative-Lanczos steps of
 * opts->dt (the restarts), each read at nfine equally spaced times from its own
 * Krylov basis (Eq. (udelta) with the fine time).  host_G[nsteps*nfine + 1] at
 * t_j = j * opts->dt / nfine receives, as kgf_greens_eq,
 *   dagger = 1: G^>(t) = -i e^{+i E0 t} <c+_a 0| e^{-iHt} |c+_a 0>,
 *   dagger = 0: G^<(t) = +i e^{-i E0 t} <c_a 0| e^{+iHt} |c_a 0>
 * (opts->direction is ignored; the retarded G(t) is G^> - G^<). */
int  kgf_greens_eq_fine(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                        const kgf_c128* psi0, double E0, int orbital, int dagger, int nsteps,
                        int nfine, const kgf_prop_opts* opts, kgf_c128* host_G);

/* kgf_fourier: host_out[j] = sum_k w_k e^{(i omega_j - eta) t_k} host_G[k],
 * t_k = k dt, trapezoid weights (dt, halved at both ends): the damped
 * transform int_0^T dt e^{i omega t - eta t} G(t) of Sec. 3 (inverse of Eq. (ft)). */
int  kgf_fourier(kgf_ctx* ctx, const kgf_c128* host_G, int nt, double dt, double eta,
                 const double* host_omega, int nw, kgf_c128* host_out);

/* ---- nonequilibrium Green's function, four-step procedure (Sec. 4) --------
 * (i)   |0> = ground state of H_ini in `sector` (kgf_ground_state, from v0)
 * (ii)  Phi(t_k) = e^{-iH t_k}|0>, t_k = k*steps_per_grid*opts->dt
 * (iii) Psi_a(t_k) = e^{+iH t_k} c_a Phi(t_k), chi_a(t_k) = e^{+iH t_k} c+_a Phi(t_k)
 * (iv)  G^<_{ab}(t,t') = i <Psi_b(t')|Psi_a(t)>, G^>_{ab}(t,t') = -i <chi_a(t)|chi_b(t')>
 * schedule 0 ("plain"): step (iii) literally, one backward run per mesh time;
 * schedule 1 ("sweep"): one backward sweep whose block grows by one column
 *   per mesh time, dotting with c_b Phi(t_s) on the way (same steps, batched);
 *   `batch` caps the block width (0 = automatic from free memory).
 * Optional zero-temperature Matsubara branch (ntau > 0) with H_ini:
 *   G^M_{ab}(+tau_j) = -<c+_a 0|e^{-(H_ini-E0)tau_j}|c+_b 0>,
 *   G^M_{ab}(-tau_j) = +<c_b 0|e^{-(H_ini-E0)tau_j}|c_a 0>,
 *   G^|_{ab}(t_k, tau_j) = i <e^{-(H_ini-E0)tau_j} c_b 0 | Psi_a(t_k)>   (= G^<(t_k, -i tau_j)),
 *   G^|_{ab}(tau_j, t_k) = -i <e^{-(H_ini-E0)tau_j} c+_a 0 | chi_b(t_k)>  (= G^>(-i tau_j, t_k)),
 *   tau_j = j * tau_steps_per_grid * dtau.
 * Outputs (host): G_lesser, G_greater [nt][nt][n_orb][n_orb] indexed (t, t');
 * G_matsubara [2][ntau][n_orb][n_orb] (+tau, -tau) or NULL; G_mixed
 * [nt][ntau][n_orb][n_orb] (t, tau) or NULL; G_mixed_left [ntau][nt][n_orb][n_orb]
 * (tau, t) or NULL; *host_E0.  If host_psi0_out is not NULL the device pointer
 * psi0_out (D) receives |0>. */
int  kgf_greens_neq(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H,
                    const kgf_sector* sector, const kgf_gs_opts* gs_opts, const kgf_c128* v0,
                    const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                    const kgf_prop_opts* opts, int schedule, int batch,
                    int ntau, int tau_steps_per_grid, double dtau,
                    kgf_c128* host_G_lesser, kgf_c128* host_G_greater,
                    kgf_c128* host_G_matsubara, kgf_c128* host_G_mixed, kgf_c128* host_G_mixed_left,
                    double* host_E0, kgf_c128* psi0_out);

/* ---- step-wise four-step run (Sec. 4, sweep schedule) ------------------------
 * The four-step G^<, G^> of kgf_greens_neq (schedule 1, no Matsubara branch),
 * run piecewise so that a caller can interleave, time or stop it.
 * kgf_neq_run_create: steps (i) and (ii) (ground state of H_ini from v0 with
 * gs_opts, forward mesh Phi(t_k) = e^{-iH t_k}|0>, t_k = k*steps_per_grid*opts->dt);
 * arguments and meanings as kgf_greens_neq.  *host_E0 receives E0.
 * kgf_neq_run_advance: runs up to n_intervals mesh intervals of steps (iii) and
 * (iv): per spin that has requested orbitals, the c sweep, then the c+ sweep,
 * each from t_max down to t_0 in chunks of source times (chunk width from
 * `batch`, else from free device memory).  One interval at mesh time t_s
 * injects c_a Phi(t_s) (c+_a Phi(t_s)) for the source times of the chunk, dots
 * every column e^{iH(t_j - t_s)} c_a Phi(t_j) of the block with c_b Phi(t_s)
 * (Sec. 4 step (iv)) and, for s > 0, moves the block to t_{s-1} by
 * steps_per_grid short-iterative-Lanczos steps (Sec. 3, Eq. (newstate)).  The
 * work is enqueued on the context's stream; the call returns once it is
 * issued (it waits for the device only when a sweep ends).  host_info (or
 * NULL) describes what ran and what comes next.
 * kgf_neq_run_result: once done, copies G^<, G^> [nt][nt][n_orb][n_orb] (host;
 * either may be NULL) -- bitwise the values of kgf_greens_neq with schedule 1
 * and the same `batch`; KGF_EINVAL while intervals are left.
 * Memory: the run owns its forward mesh, sweep block and G until
 * kgf_neq_run_destroy (other calls on the context may run in between and do
 * not touch them); the context, models and sector must outlive the run.
 * KGF_ENOCONV from create if the ground state does not converge. */
typedef struct kgf_neq_run kgf_neq_run;
typedef struct {
    int     intervals;           /* mesh intervals run by this call                       */
    int     width;               /* block columns of the last interval run                */
    int     done;                /* 1 when every sweep has finished                       */
    int     next_width;          /* block columns of the next interval (0 when done)      */
    int     next_mesh_index;     /* mesh index s of the next interval (-1 when done)      */
    int     chunk_width;         /* full block width of the next interval's chunk         */
    int     branch;              /* index of the next interval's sweep (order above), -1 when done */
    int64_t vector_steps;        /* single-column SIL steps run by this call              */
    int64_t total_vector_steps;  /* single-column SIL steps since creation                */
    int     chunk_start;         /* 1 when the next interval begins a chunk, or when done
                                    (where kgf_neq_run_checkpoint may be called)          */
} kgf_neq_run_info;
int  kgf_neq_run_create(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H, const kgf_sector* sector,
                        const kgf_gs_opts* gs_opts, const kgf_c128* v0, const int32_t* host_orbs, int n_orb,
                        int nt, int steps_per_grid, const kgf_prop_opts* opts, int batch,
                        kgf_neq_run** out, double* host_E0);
int  kgf_neq_run_advance(kgf_neq_run* run, int n_intervals, kgf_neq_run_info* host_info);
int  kgf_neq_run_result(kgf_neq_run* run, kgf_c128* host_G_lesser, kgf_c128* host_G_greater);
void kgf_neq_run_destroy(kgf_neq_run* run);

/* Checkpoint and resume of a step-wise run (host spill).  The forward mesh
 * Phi(t_k) of Sec. 4 step (ii) is recomputed from the same inputs, so an
 * image holds only the progress of steps (iii)-(iv): the position of the
 * backward sweeps, the dot products of Sec. 4 step (iv) placed so far for the
 * current sweep and G^<, G^> of the finished sweeps (nt^2 n_orb^2 complex
 * numbers each, plus nt^2 n^2 for the current sweep's n orbitals).
 * kgf_neq_run_checkpoint: writes the image into host_buf (host memory of
 * `bytes` bytes, owned by the caller) and its size into *host_bytes_needed
 * (may be NULL); with host_buf NULL only the size is reported.  Valid between
 * chunks, i.e. when the next interval starts a chunk or the run is done
 * (kgf_neq_run_info::chunk_start == 1); KGF_EINVAL inside a chunk or for a
 * short buffer.  The call waits for the run's device work.
 * kgf_neq_run_restore: on a run just created (no kgf_neq_run_advance yet) from
 * the same models, sector, v0, orbitals and options, loads an image; the run
 * then continues where the saved one stopped, the current sweep with the
 * saved chunk length, so that its result equals the uninterrupted run's
 * bitwise when `batch` is given (otherwise later sweeps size their chunks
 * from the free memory of this run).  KGF_EINVAL for an image of another run
 * (sizes, or a ground-state energy that differs by more than 1e-12
 * relative), a run that has advanced, or a damaged image. */
int  kgf_neq_run_checkpoint(kgf_neq_run* run, void* host_buf, size_t bytes, size_t* host_bytes_needed);
int  kgf_neq_run_restore(kgf_neq_run* run, const void* host_buf, size_t bytes);

/* Four-step G^< and G^> (Sec. 4 steps (i)-(iv), sweep schedule) of n_inst
 * independent instances in one call.  Instances whose sectors have equal
 * (L, N_up, N_dn) and whose H have the same bond list form a group that runs
 * as one batch: every Lanczos / SIL launch of the forward meshes and the
 * backward sweeps serves all members, column c carrying the parameters of
 * member c mod n (different hoppings, on-site energies and U per instance);
 * with KGF_OPT_LOCKSTEP (default) the groups themselves advance together,
 * each kernel of a SIL step one launch over every group's columns;
 * ground states are found one instance at a time.  Results equal
 * kgf_greens_neq on each instance up to rounding.
 * Per-instance inputs: H_ini[i], H[i], sectors[i], v0[i] (device, D_i).
 * Outputs (host): host_G_lesser, host_G_greater [n_inst][nt][nt][n_orb][n_orb]
 * (NULL to skip); host_E0 [n_inst].  `batch` caps the columns of one sweep
 * block (0 = from free memory).  No Matsubara branch.  Errors as kgf_greens_neq. */
int  kgf_greens_neq_multi(kgf_ctx* ctx, int n_inst, const kgf_model* const* H_ini,
                          const kgf_model* const* H, const kgf_sector* const* sectors,
                          const kgf_c128* const* v0, const kgf_gs_opts* gs_opts,
                          const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                          const kgf_prop_opts* opts, int batch, kgf_c128* host_G_lesser,
                          kgf_c128* host_G_greater, double* host_E0);

/* ---- parameter derivatives and the adjoint (reverse mode) ------------------
 * Parameters of a model: theta = (t_b for b < n_bonds, eps_up_i, eps_dn_i,
 * U_i for i < L), n_theta = n_bonds + 3 L; dH/dt_b = -sum_s (c+_i c_j + h.c.),
 * dH/deps_is = n_is, dH/dU_i = n_i,up n_i,dn (the H of the header comment).
 * Cotangents follow psi_bar = dL/d(psi*) for a real loss L, so that
 * dL = 2 Re <psi_bar|d psi>; for G, W is the cotangent with
 * dL = Re sum conj(W) dG (W = 2 dL/dG* for a loss written in G, G*). */
int  kgf_n_theta(const kgf_model* model);

/* host_grad[theta] = sum_p Re( host_w[p] <lam_p| dH/dtheta |psi_p> ), for npair
 * vector pairs at lam + p*ld, psi + p*ld (device).  host_grad has n_theta
 * doubles and is overwritten. */
int  kgf_dH_expect(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                   const kgf_c128* lam, const kgf_c128* psi, int npair, int64_t ld,
                   const kgf_c128* host_w, double* host_grad);

/* Adjoint of kgf_propagate for one vector (direction -1 or +1): psi0 is the
 * initial state (device, D, unchanged); lam enters as the cotangent of the
 * state after nsteps steps and leaves as the cotangent of psi0.  host_grad
 * (n_theta doubles, overwritten) receives dL/dtheta of the propagation:
 * per step 2 Re[ dir i int_0^dt <lam(s)| dH/dtheta |psi(s)> ds ] (derivative of
 * the propagator, Sec. 3 Eq. (newstate) taken as exact), the integral by
 * quad_nodes-point Gauss-Legendre with the node states from each step's own
 * Krylov spaces (fine-grid evaluation, Eq. (udelta)).  Workspace: nsteps
 * vectors (the recomputed chain) plus 2 quad_nodes node vectors. */
int  kgf_propagate_vjp(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* sector,
                       const kgf_c128* psi0, kgf_c128* lam, int nsteps, const kgf_prop_opts* opts,
                       int quad_nodes, double* host_grad);

/* Gradient of L = Re sum conj(W^<) G^< + Re sum conj(W^>) G^> for the
 * four-step G of kgf_greens_neq (plain schedule; same arguments and
 * layouts), with respect to the parameters of H (host_grad) and of H_ini
 * (host_grad_ini, through the ground state: d|0> = -(H_ini - E0)^+ (1 - P0)
 * dH_ini |0>, solved by projected conjugate gradients to relative residual
 * cg_tol).  host_W_lesser / host_W_greater: [nt][nt][n_orb][n_orb] or NULL
 * (zero).  Optional outputs: G^<, G^> of the forward pass, E0, the number
 * of CG iterations.  Cost: about four forward passes; memory: the forward
 * mesh, the backward-propagated states of every mesh time and one chain.
 * KGF_ENOCONV (outputs still written, host_grad_ini not to be trusted) when
 * the projected CG stops above cg_tol: at its iteration limit
 * (KGF_OPT_CG_MAX_ITER) or on a non-positive curvature p^T (H - E0) p, which
 * a (near-)degenerate ground state produces. */
int  kgf_greens_neq_vjp(kgf_ctx* ctx, const kgf_model* H_ini, const kgf_model* H,
                        const kgf_sector* sector, const kgf_gs_opts* gs_opts, const kgf_c128* v0,
                        const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                        const kgf_prop_opts* opts, const kgf_c128* host_W_lesser,
                        const kgf_c128* host_W_greater, int quad_nodes, double cg_tol,
                        double* host_grad_ini, double* host_grad, kgf_c128* host_G_lesser,
                        kgf_c128* host_G_greater, double* host_E0, int* host_cg_iters);

/* Gradients of kgf_greens_neq_vjp for n_inst instances in one call.
 * Instances whose sectors have equal (L, N_up, N_dn) and whose H have the
 * same bond list form a group whose propagations, chain adjoints and adjoint
 * steps run as one batch (column c carries member c mod n); ground states,
 * Gram matrices and the ground-state solves are per instance.  Results equal
 * kgf_greens_neq_vjp on each instance up to rounding.  Per-instance arrays:
 * H_ini[i], H[i], sectors[i], v0[i] (device), host_W_lesser[i] /
 * host_W_greater[i] (host [nt][nt][n_orb][n_orb]; the arrays of pointers may
 * be NULL, entries NULL = zero cotangent), host_grad_ini[i] (n_theta(H_ini[i])
 * doubles), host_grad[i] (n_theta(H[i]) doubles; NULL entries skip);
 * host_E0 [n_inst]; host_cg_iters [n_inst] or NULL.  Memory: the plain-
 * schedule meshes of kgf_greens_neq_vjp times the group size.  KGF_ENOCONV
 * as kgf_greens_neq_vjp when the CG of any instance stops above cg_tol. */
int  kgf_greens_neq_vjp_multi(kgf_ctx* ctx, int n_inst, const kgf_model* const* H_ini,
                              const kgf_model* const* H, const kgf_sector* const* sectors,
                              const kgf_gs_opts* gs_opts, const kgf_c128* const* v0,
                              const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                              const kgf_prop_opts* opts, const kgf_c128* const* host_W_lesser,
                              const kgf_c128* const* host_W_greater, int quad_nodes, double cg_tol,
                              double* const* host_grad_ini, double* const* host_grad,
                              double* host_E0, int* host_cg_iters);

/* ---- progress reporting ------------------------------------------------------
 * The drivers (kgf_ground_state, kgf_greens_eq, kgf_greens_neq) call
 * fn(user, phase, done, total) on the calling host thread after each mesh
 * time (and at phase boundaries), once the work up to that point has
 * finished on the device.  `phase` is a short static string.  fn = NULL
 * disables reporting (the default).  The callback must not call back into
 * the library. */
typedef void (*kgf_progress_fn)(void* user, const char* phase, int64_t done, int64_t total);
int  kgf_set_progress(kgf_ctx* ctx, kgf_progress_fn fn, void* user);

/* ---- kernel-variant options ---------------------------------------------------
 * Choices between equivalent kernels (results agree to rounding).  By default
 * the library picks by the sector's sizes.
 *   KGF_OPT_HV_PASSES: 0 by size; 1 single-pass H.v (source row staged in LDS,
 *                      rows up to 78 KB only); 2 two-pass H.v (pass 1: row in
 *                      LDS, down-spin hops and diagonal; pass 2: up-spin hops on
 *                      L2-sized column strips); 3 two-pass with rows staged as
 *                      real and imaginary halves (the mode used for rows above
 *                      78 KB); 4 two-pass with one whole row per pass-1 block
 *                      (2 and 3 stage two rows per block where they fit).
 *   KGF_OPT_HV_STRIP:  0 by size (the widest of 64, 32, 16, 8 that the rows
 *                      fill), or 8, 16, 32, 64, 128 columns per strip (pass 2).
 *   KGF_OPT_GS_MAX_BASIS: 0 = the ground-state Lanczos basis holds up to
 *                      max_iter + 1 vectors if they fit in 70% of free device
 *                      memory; n >= 8 caps it at n vectors.  Below max_iter + 1
 *                      the recursion restarts from the current Ritz vector every
 *                      n - 1 steps (same stopping rule, more iterations).
 *   KGF_OPT_PHI_EVERY: 0 = kgf_greens_neq stores the forward mesh Phi(t_k) whole
 *                      if it takes at most 35% of free device memory, else keeps
 *                      every K-th state (smallest K whose checkpoints and one
 *                      recomputed segment take at most 30%); n >= 1 fixes K = n.
 *                      Recomputed states are bitwise equal to stored ones.
 *   KGF_OPT_ADJ_EVERY: 0 = the adjoints (kgf_propagate_vjp, kgf_greens_neq_vjp)
 *                      store the states of each propagation chain whole if they
 *                      take at most 30% of free device memory, else keep every
 *                      K-th state and recompute one segment at a time;
 *                      n >= 1 fixes K = n (checkpoint every n SIL steps).
 *   KGF_OPT_HV_TUNE:   0 (default) = H.v variant by size; 1 = the first H.v of
 *                      each sector (L, N_up, N_dn) times every equivalent variant
 *                      (single pass, two pass with strips 16/32/64, split rows)
 *                      on scratch vectors, separately for the plain form (three
 *                      H.v) and the Lanczos form (one SIL step of Krylov
 *                      dimension 20 on one column, the update pass or the
 *                      folded update included), and keeps the fastest for that
 *                      context;
 *                      and the four-step sweeps with batch = 0 time one SIL
 *                      step per block width (the widest that fits, 32, 16, 8, 4
 *                      columns) on scratch columns of the target sector and keep
 *                      the width with the most column-steps per second (cached
 *                      per sector and Krylov options; columns do not depend on
 *                      the width).  HV_PASSES / HV_STRIP, when set, take precedence.
 *   KGF_OPT_CG_MAX_ITER: iteration limit of the projected CG of the four-step
 *                      adjoints (0 = 20000).
 *   KGF_OPT_GRAPHS:    1 = a batched SIL step that recurs with the same model
 *                      parameters, sector, state buffer, batch width and options
 *                      (the steps of one kgf_propagate call, the intervals of a
 *                      four-step sweep) is captured once in a hipGraph and
 *                      replayed (the same kernels and arguments: bitwise the eager
 *                      results); not while kgf_profile_begin is active.  0
 *                      (default) = eager: a SIL step is a few dozen launches of
 *                      0.1-15 ms, whose launch cost the stream already hides.
 *                      Changing any option drops the captured steps.
 *   KGF_OPT_LOCKSTEP:  1 (default) = kgf_greens_neq_multi advances the groups of
 *                      instances with small sectors (at most 2^17 states) together:
 *                      every kernel of a SIL step is one launch over the columns of
 *                      all of them (sectors of different size, a Hamiltonian per
 *                      column; the H.v one launch per row block size), the sweeps
 *                      share one chunk of source times; larger sectors fill the GPU
 *                      alone and run group by group.  Same results as group by group
 *                      (per group the same element owners and reduction orders).
 *                      Used when reorth = 0 and those sectors' H.v is the single
 *                      pass; 0 = every group alone.
 *   KGF_OPT_HV_FUSE:   1 (default) = where a sector's H.v is two-pass and
 *                      reorth = 0, a Lanczos step (Eq. (recursion)) is the two
 *                      passes alone: the update y - a_k v_k of step k and the
 *                      norm giving b_{k+1} are done by the row pass of step k+1
 *                      while it stages those rows (no separate update pass);
 *                      0 = the update as a pass of its own.  Results agree to
 *                      rounding.
 *   KGF_OPT_HV_SEG:    1 (default) = pass 1 of the two-pass H.v finds the
 *                      down-spin hops from segment tables: the masks split into
 *                      a high and a low half, a hop inside one half moves the
 *                      rank by an offset that depends on that half alone (tens
 *                      of KB of tables in LDS instead of one table entry per
 *                      state and hop); used when at most 8 bonds cross the
 *                      split and the row and tables fit in LDS.  0 = the
 *                      per-state tables.  Results agree to rounding.
 *   KGF_OPT_HV_UP_THREADS: threads per block of pass 2 of the two-pass H.v
 *                      (256, 512 or 1024 = default; a block covers threads / C
 *                      rows of one strip).  Results are independent of it.
 * Returns KGF_EINVAL for an unknown option or value.  Not to be changed while
 * work issued by this context is in flight. */
enum { KGF_OPT_HV_PASSES = 1, KGF_OPT_HV_STRIP = 2, KGF_OPT_GS_MAX_BASIS = 3, KGF_OPT_PHI_EVERY = 4, KGF_OPT_ADJ_EVERY = 5,
       KGF_OPT_HV_TUNE = 6, KGF_OPT_CG_MAX_ITER = 7, KGF_OPT_GRAPHS = 8, KGF_OPT_LOCKSTEP = 9,
       KGF_OPT_HV_FUSE = 10, KGF_OPT_HV_SEG = 11, KGF_OPT_HV_UP_THREADS = 12 };
int  kgf_set_option(kgf_ctx* ctx, int option, int value);

/* ---- device-side timing of the library's kernels --------------------------
 * Between kgf_profile_begin and kgf_profile_end every `sample_every`-th
 * launch of each kernel class is bracketed by HIP events on the context's
 * stream.  kgf_profile_end synchronises and fills up to max_classes rows:
 * class name (<= 31 chars), launches, sampled launches, summed sampled
 * milliseconds and the summed algorithmic bytes of the sampled launches
 * (the minimum HBM traffic of each launch: every input vector read once,
 * every output vector written once; 0 for classes without a byte model).
 * Returns the number of classes written (>= 0). */
typedef struct {
    char   name[32];
    int64_t launches;
    int64_t sampled;
    double sampled_ms;
    double sampled_bytes;
} kgf_kernel_stat;
int  kgf_profile_begin(kgf_ctx* ctx, int sample_every);
int  kgf_profile_end(kgf_ctx* ctx, kgf_kernel_stat* host_stats, int max_classes);

#ifdef __cplusplus
}
#endif
#endif /* KGF_H */
