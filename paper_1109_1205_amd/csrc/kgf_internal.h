// Internal declarations of libkgf (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kgf.h"

namespace kgf {

// Internal failures travel as exceptions and are turned into return codes
// at the ABI boundary (api.hip); none crosses the C interface.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

#define KGF_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            ::kgf::fail(KGF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define KGF_REQUIRE(cond, code, msg)                                           \
    do {                                                                       \
        if (!(cond)) ::kgf::fail((code), (msg));                               \
    } while (0)

constexpr int kMaxL = 24;          // masks are uint32; column ranks need 24 bits
constexpr int kMaxBonds = 127;     // bond index stored in 7 bits
constexpr int kMaxKrylov = 128;    // SIL Krylov dimension (one or two wavefronts per tridiagonal matrix)
constexpr int kBinomN = 33;        // binomial table C[n][k], n,k < 33
constexpr int kThreads = 256;      // threads per block of the streaming kernels

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void reserve(size_t n);          // discards contents when it grows
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Segment form of one spin species' hopping for n particles (built on the
// host with the hopping table, hamiltonian.hip build_seg_table).  A mask s
// is split at bit S into its high part H = s >> S and low part l = s &
// (2^S - 1); in ascending mask order the states with one H are contiguous
// (a segment of C(S, n - |H|) states, ascending in l).  A hop on a bond
// inside the low part moves the rank by rank_lo(l') - rank_lo(l), a function
// of l alone; a hop inside the high part by seg_off(H') - seg_off(H), a
// function of H alone; a hop on a bond across the split by the sum of one
// low and one high part.  One packed table of 32-bit words (tens of KB)
// replaces the per-state ELL entries.
struct SegInfo {
    int S = -1;            // split bit; -1 = not built, 0 = not usable
    int nl = 0, nh = 0;    // 2^S, 2^(L-S)
    int wlo = 0, whi = 0;  // entry slots per low / high part (padded)
    int ncross = 0;        // bonds across the split
    int words = 0;         // packed table size (32-bit words)
    // word offsets.  lo [wlo][nl] (indexed by the low part's position p in
    // (popcount, rank) order) and hi [whi][nh]: delta << 9 | amplitude slot,
    // delta a signed rank offset, slot 2 bond + sign (256: padding, zero);
    // cl [ncross][nl] (by p) and ch [ncross][nh]: delta << 2 | occupied << 1 |
    // parity of the occupied sites between; seg [nh] (int32 segment offsets,
    // -1 where H has no segment); cls [S + 2] (first position of each
    // popcount); cbond [ncross] (bond index)
    int o_lo = 0, o_hi = 0, o_cl = 0, o_ch = 0, o_seg = 0, o_cls = 0, o_cbond = 0;
};

// Per-spin tables of one particle number n for one model (hopping matrix
// in ELL layout plus the on-site energy of each mask for either spin).
struct HopTable {
    int n = 0;
    int64_t D = 0;
    int width = 0;
    DevBuf masks;    // uint32 [D]
    DevBuf count;    // int32  [D]
    DevBuf ent;      // uint32 [width * D]
    DevBuf e_up;     // double [D]  sum_i eps_up[i] bit_i
    DevBuf e_dn;     // double [D]  sum_i eps_dn[i] bit_i
    DevBuf bond;     // uint32 [nb * D] per bond: target rank | sign << 31, or ~0u
    DevBuf order;    // int32  [D] ranks grouped by the popcount of the mask's upper
                     // half (L/2 and up), ascending within a group: the row order
                     // of the up-spin strip pass of the two-pass H.v
    SegInfo seg;     // segment form (seg_table)
    DevBuf segtab;   // its packed words
};

struct KernelStat {
    int64_t launches = 0;
    int64_t sampled = 0;
    double ms = 0.0;
    double bytes = 0.0;
};

}  // namespace kgf

struct kgf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    kgf::DevBuf binom;                       // uint64 [kBinomN * kBinomN]
    std::map<std::string, std::unique_ptr<kgf::DevBuf>> ws;
    // profiling
    bool prof_on = false;
    int prof_every = 1;
    std::map<std::string, kgf::KernelStat> prof;
    struct Pending { std::string name; hipEvent_t a, b; double bytes; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    // H.v variant knobs (kgf_set_option)
    int hv_passes = 0;
    int hv_strip = 0;
    int gs_max_basis = 0;                    // 0: as many Lanczos vectors as fit
    int phi_every = 0;                       // 0: forward mesh stored whole when it fits
    int adj_every = 0;                       // 0: adjoint chains stored whole when they fit
    int hv_tune = 0;                         // 1: time the H.v variants of each sector once
    int cg_max_iter = 0;                     // 0: 20000 (projected CG of the adjoints)
    // captured SIL steps (hipGraph), replayed when the same step recurs
    int use_graphs = 0;
    int lockstep = 1;                        // 1: uneven instance groups advance together (grouped launches)
    int hv_fuse = 1;                         // 1: two-pass Lanczos steps fold the update into pass 1
    int hv_seg = 1;                          // 1: pass 1 of the two-pass H.v uses the segment hop tables
    int hv_up_threads = 1024;                // block size of pass 2 of the two-pass H.v (256, 512, 1024)
    struct SilGraph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
        uint64_t last_use = 0;
    };
    std::vector<SilGraph> sil_graphs;
    uint64_t graph_clock = 0;
    hipStream_t capture_stream = nullptr;
    // host copies of the device tables of the last grouped launch
    std::vector<unsigned char> hvg_table, gcol_table;
    // pinned staging ring for small table uploads (stream-ordered, no host wait)
    static constexpr int kStageSlots = 4;
    void* stage[kStageSlots] = {};
    size_t stage_bytes[kStageSlots] = {};
    hipEvent_t stage_ev[kStageSlots] = {};
    int stage_next = 0;
    std::map<std::array<int, 4>, std::pair<int, int>> hv_tuned;   // (L, N_up, N_dn, mode) -> (passes, strip)
    std::map<std::array<int, 4>, int> sweep_tuned;                // (L, 64 N_up + N_dn, m, reorth) -> columns
    // progress callback
    kgf_progress_fn progress = nullptr;
    void* progress_user = nullptr;
    // pinned host scratch for scalar readbacks
    void* host_scratch = nullptr;
    size_t host_scratch_bytes = 0;
};

struct kgf_model {
    kgf_ctx* ctx = nullptr;
    uint64_t version = 0;  // unique per creation and per parameter change (keys of captured steps)
    int L = 0;
    int nb = 0;
    std::vector<int32_t> bi, bj;
    std::vector<double> t, eps_up, eps_dn, U;
    bool U_uniform = true;
    kgf::DevBuf d_t;       // double [nb]  hopping amplitudes
    kgf::DevBuf d_Utab;    // double [3 * 256] sum of U_i over the set bits of each mask byte
    std::map<int, std::unique_ptr<kgf::HopTable>> tables;
};

struct kgf_sector {
    kgf_ctx* ctx = nullptr;
    int L = 0, n_up = 0, n_dn = 0;
    int64_t d_up = 0, d_dn = 0;
    kgf::DevBuf masks_up, masks_dn;   // uint32
    int64_t dim() const { return d_up * d_dn; }
};

namespace kgf {

// ---- context helpers (api.hip) -------------------------------------------
void* workspace(kgf_ctx* ctx, const std::string& name, size_t bytes);
void* host_scratch(kgf_ctx* ctx, size_t bytes);
void sync(kgf_ctx* ctx);
void check_launch(const char* what);
void ensure_device_fits(size_t bytes, const char* what);
// report progress (synchronises the stream first; no-op without a callback)
void progress(kgf_ctx* ctx, const char* phase, int64_t done, int64_t total);

// RAII bracket of one kernel launch for kgf_profile_*; `bytes` is the
// launch's algorithmic HBM traffic (0 when not modelled).
struct Prof {
    kgf_ctx* ctx;
    const char* name;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Prof(kgf_ctx* c, const char* n, double bytes = 0.0);
    ~Prof();
};

// copy n bytes of host data into the device workspace `name` in stream
// order through the pinned staging ring (the host does not wait for the
// stream); returns the device pointer
void* upload_table(kgf_ctx* ctx, const std::string& name, const void* host, size_t n);

// unique version stamps of models and model sets
uint64_t next_version();
// forget every captured SIL step of the context (waits for the stream)
void drop_graphs(kgf_ctx* ctx);

// ---- basis (basis.hip) ----------------------------------------------------
void build_binomials(kgf_ctx* ctx);
void build_masks(kgf_ctx* ctx, int L, int n, uint32_t* masks, int64_t D);
void rank_masks(kgf_ctx* ctx, const uint32_t* masks, int64_t n, int N, int64_t* ranks);
int64_t binom_host(int n, int k);

// ---- hamiltonian (hamiltonian.hip) ---------------------------------------
HopTable& hop_table(kgf_model* model, int n);
// device copies of a model's hopping amplitudes and U byte tables
void upload_params(kgf_model* m);
// after a parameter change: recompute the on-site energies of the built tables
void refresh_onsite(kgf_model* model);
// segment form of a spin species' hopping (built with its hopping table)
const SegInfo& seg_table(kgf_model* model, int n);
void build_seg_table(kgf_model* model, HopTable& ht);
// replace a model's parameters in place (same L and bonds); waits for the
// context's stream first, so that work already issued keeps the old values
void model_set_params(kgf_model* m, const double* t, const double* eps_up, const double* eps_dn,
                      const double* U);

// Drive of H(t) = sum_j f_j(t) H_j: theta[j * n_theta(work) ..] = parameters
// of H_j; f[(n * 2 + q) * n_terms + j] = f_j at Gauss node q of step n.
struct DriveTable {
    int n_terms;
    const double* theta;
    const double* f;
};
// set `work` to the Hamiltonian of stage s (0: B_1, 1: B_2) of step n of the
// fourth-order commutator-free integrator (driven.hip)
void driven_stage(kgf_model* work, const DriveTable& drv, int n, int stage);

// Parameter sets of several models with one bond topology (same L and bond
// list), for batches whose columns carry different Hamiltonians: column c
// of a launch uses member c mod n.  The hopping tables (targets, bonds,
// signs) depend on the topology only and are shared.
struct ModelSet {
    uint64_t version = 0;  // unique per model_set_init
    std::vector<kgf_model*> models;
    bool U_uniform = true;
    DevBuf t;      // double [n][nb]
    DevBuf Utab;   // double [n][3 * 256]
    DevBuf U0;     // double [n]
    std::map<int, std::unique_ptr<DevBuf>> eu, ed;   // by particle number: double [n][D_n]
};
void model_set_init(kgf_ctx* ctx, ModelSet& set);   // checks the topology, uploads t, U
bool same_topology(const kgf_model* a, const kgf_model* b);

// What H.v needs: one model, or a model set (one member per column).
struct HModel {
    kgf_model* m = nullptr;
    ModelSet* set = nullptr;
    HModel(kgf_model* mm) : m(mm) {}
    explicit HModel(ModelSet* s) : m(s->models.at(0)), set(s) {}
};

void apply_h(kgf_ctx* ctx, HModel model, const kgf_sector* sec,
             const double2* v, double2* w, int nvec, int64_t ld);
// With ctx->hv_tune set, times the equivalent H.v variants of the sector once
// (plain and Lanczos forms; the Lanczos form separately for one column and,
// when ncol > 1, for several) and keeps the fastest; a no-op otherwise.
void hv_prepare(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int ncol = 1);
void apply_c(kgf_ctx* ctx, const kgf_sector* src, const kgf_sector* dst, int orbital,
             int dagger, const double2* v, double2* w, int nvec, int64_t ld_src,
             int64_t ld_dst);

// Parameter derivatives of H: theta = (t_b [nb], eps_up [L], eps_dn [L], U [L]);
// dH/dt_b = -K_b (K_b = sum_s c+_i c_j + h.c.), dH/deps_is = n_is,
// dH/dU_i = n_i,up n_i,dn.  Adds Re(w * <lam| dH/dtheta |psi>) to g[theta]
// (device, n_theta doubles) for each of npair pairs (lam_p, psi_p, w_p).
int n_theta(const kgf_model* model);
void dH_expect(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* lam,
               int64_t lam_col, const double2* psi, int64_t psi_col, int npair,
               const double2* host_w, double* g);

// Lanczos-fused H.v: for each column c
//   y_c = s_c[k] * H x_c - b_c[k] * s_c[k-1] * xp_c      (xp may be null)
//   part[c][blk] = Re <s_c[k] x_c, y_c>   (one partial per block)
struct LanczosHvArgs {
    const double2* x; int64_t x_col;       // x_c = x + c * x_col
    const double2* xp; int64_t xp_col;     // previous vector (nullable)
    double2* y; int64_t y_col;
    const double* s_k;                     // scale of x (per column, * stride)
    const double* b_k;                     // b_k       (per column, * stride)
    const double* s_km1;                   // scale of xp (per column, * stride)
    int stride;                            // doubles between columns
    double* part;                          // [ncol][nblk]
};
int hv_lanczos_blocks(kgf_ctx* ctx, const kgf_sector* sec);
// partials per column a Lanczos step may write (either pass of a fused step)
int hv_part_capacity(kgf_ctx* ctx, const kgf_sector* sec);
void hv_lanczos(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int ncol,
                const LanczosHvArgs& a);

// Two-pass Lanczos step with the update of the previous step folded into
// pass 1 (sectors whose H.v plan is two-pass).  Step k is
//   rows: x_k = y - a_{k-1} s_{k-1} x_{k-1} written back over y (slot k),
//         part[c][blk] = partials of ||x_k||^2 (-> b_k, s_k), and
//         z = (down-spin hops + diagonal) x_k;  for k = 0 (xp null) x_0 is
//         the state itself, read only;
//   up:   y = s_k (z + T_up x_k) - b_k s_{k-1} x_{k-1} in place of z,
//         part = Re <s_k x_k, y> (-> a_k)   (hv_lanczos_up with y = z).
// The separate update pass (y -= a_k v_k, ||y||^2) is not needed: the rows
// pass reads the rows it would touch anyway.
struct LanczosRowsArgs {
    double2* x; int64_t x_col;             // slot k (y in, x_k out when xp is set)
    double2* z; int64_t z_col;             // pass-1 output (slot k + 1)
    const double2* xp; int64_t xp_col;     // x_{k-1}, null for k = 0
    const double* fa;                      // a_{k-1} (per column, * stride)
    const double* fs;                      // s_{k-1}
    int stride;
    double* part;                          // [ncol][hv_lanczos_rows_blocks]
};
// Pass-1 blocks (norm partials) per column of a fused step over ncol
// columns; 0 when that step is not two-pass.  up_blocks (if given) receives
// the pass-2 partials per column.  Where the rows fit the single pass, the
// fused two-pass step is chosen for launches whose columns together exceed
// the Infinity Cache: the single pass's separate update pass then streams
// from HBM instead of finding the vector it just wrote in that cache.
int hv_lanczos_rows_blocks(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int ncol, int* up_blocks = nullptr);
void hv_lanczos_rows(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int ncol, const LanczosRowsArgs& a);
void hv_lanczos_up(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int ncol, const LanczosHvArgs& a);

// ---- krylov (krylov.hip) -------------------------------------------------
// Per-column scalar block of the SIL recursion (doubles): offsets of b_k and
// s_k (the full layout lives in krylov.hip).
constexpr int kScalOffB = 128;
constexpr int kScalOffS = 258;

// One column of a launch that serves several instance groups: its Krylov
// slots (slot 0 is the state), dimension, partial-sum area and group.
struct GroupCol {
    double2* s0;
    double2* X1;
    int64_t x_slot;
    int64_t D;
    double* part;
    int group;
    int nb;            // blocks per column of the streaming kernels
    int nrow;          // rows (D_up): partials of the Lanczos H.v
    __host__ __device__ double2* at(int k) const { return k == 0 ? s0 : X1 + (int64_t)(k - 1) * x_slot; }
};

// Block range of one group in a flattened grouped launch: global blocks
// [blk0, blk0 + nb * ncol) serve columns col0.. with nb blocks each.
struct GroupRange {
    int64_t blk0;
    int nb;
    int col0;
};
// group, column and block within the column of flattened block b
__device__ __forceinline__ int group_of_block(const GroupRange* r, int ng, int64_t b) {
    int g = 0;
    while (g + 1 < ng && b >= r[g + 1].blk0) ++g;
    return g;
}

// An instance group of a grouped launch: its model (or model set), sector
// and global columns [col0, col0 + ncol).
struct GroupSpec {
    HModel model;
    const kgf_sector* sec;
    int col0;
    int ncol;
};
// true when every group's Lanczos H.v is the single pass (rows in LDS)
bool hv_groups_supported(kgf_ctx* ctx, const std::vector<GroupSpec>& groups);
// Lanczos-fused H.v of step k for every column of every group in one launch
// (cols: device descriptors, scal: per-column scalar blocks of stride stride)
void hv_lanczos_groups(kgf_ctx* ctx, const std::vector<GroupSpec>& groups, const GroupCol* cols, int ncol_total,
                       int k, const double* scal, int stride);
// flattened grid of 1D blocks over n blocks (x up to 2^31 - 1, then y)
inline dim3 flat_grid(int64_t n) {
    const int64_t x = n < 0x7fffffff ? n : 0x7fffffff;
    return dim3((unsigned)(x > 0 ? x : 1), (unsigned)((n + x - 1) / (x > 0 ? x : 1)));
}
__device__ __forceinline__ int64_t flat_block() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

struct SilOpts {
    int m;
    int reorth;
    double dt;
    int direction;
    double shift;
    double breakdown_tol;
};

// Reserve the SIL workspaces for batches of up to ncol columns (avoids
// re-allocation when a caller grows its batch step by step).
void sil_reserve(kgf_ctx* ctx, const kgf_sector* sec, int ncol, int m, int reorth);
// Lanczos bases of ncol columns (slot 0 = psi + c*ld), left in the SIL workspace.
void sil_build(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi, int ncol,
               int64_t ld, const SilOpts& o);
// Coefficients of exp(dir i H t) (or exp(-(H - shift) t) for dir 0) applied to
// column col[r], in the basis of the last sil_build: coef + r * coef_stride.
void sil_coefs(kgf_ctx* ctx, int m, int nreq, const int* col, const double* t, const int* dir,
               double shift, double2* coef, int coef_stride);
// out + o * out_col = sum_j coef[o][j] v_j(column c), o < nout (one pass over the basis)
void sil_combine_multi(kgf_ctx* ctx, const kgf_sector* sec, double2* psi, int64_t ld, int ncol, int m,
                       int c, const double2* coef, int64_t coef_stride, int nout, double2* out,
                       int64_t out_col);
// Batched short-iterative-Lanczos step(s) on ncol columns psi_c = psi + c*ld.
// err (device, ncol doubles, or null): the largest a-posteriori step error
// estimate of each column over the steps; drift (device, ncol doubles, or
// null): the largest | ||psi after|| / ||psi before|| - 1 | of each column
// over the steps (one norm pass per step).
void sil_propagate(kgf_ctx* ctx, HModel model, const kgf_sector* sec, double2* psi,
                   int ncol, int64_t ld, int nsteps, const SilOpts& o, double* err = nullptr,
                   double* drift = nullptr);

// Bytes of the one buffer that sil_propagate_in carves its Krylov slots,
// scalars and partials from, and SIL steps with every device buffer in
// `scratch` (no allocation; the model's hopping tables for the sector's
// particle numbers must exist).
size_t sil_scratch_bytes(kgf_ctx* ctx, const kgf_sector* sec, int ncol, int m, int reorth);
// Returns the device address of the per-column error estimates when
// want_err (inside the scratch), else null.
double* sil_propagate_in(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, double2* psi, int ncol, int64_t ld,
                         int nsteps, const SilOpts& o, void* scratch, bool want_err);
// true when the model's hopping table for n particles has been built
bool hop_table_ready(const kgf_model* model, int n);

struct GsResult {
    double E0;
    int iters;
    bool converged;
    double residual;
};
GsResult ground_state(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec,
                      const double2* v0, double2* psi0, double tol, int max_iter,
                      int check_every, int reorth);

// v[i] = SplitMix64 output i of `seed` mapped to [-1, 1) (real), i < n
void fill_splitmix(kgf_ctx* ctx, double2* v, int64_t n, uint64_t seed);
// sweep block width chosen by timing one SIL step per candidate width (cached
// per sector shape and Krylov options; at most max_cols)
int tuned_sweep_width(kgf_ctx* ctx, HModel model, const kgf_sector* sec, int max_cols, const SilOpts& o);
// drop a workspace (waits for the stream first)
void release_ws(kgf_ctx* ctx, const char* name);

// |<psi0|psi_b>|^2 for psi_b the ground state from a second (SplitMix64) start
// vector, and the check that raises KGF_EDEGENERATE below 1 - unique_tol
// (no-op unless o->unique_check).
double gs_fidelity2(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0,
                    const kgf_gs_opts* o);
void require_unique_ground_state(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0,
                                 const kgf_gs_opts* o, const char* who);

// n Lanczos steps from i0: a[0..n), b[1..n) (host), <i0|i0>; returns the
// steps taken (fewer when the Krylov space is exhausted).
int lanczos_tridiag(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* i0, int n, int reorth,
                    double* a_host, double* b_host, double* norm2_host);

// G[l][r] = <L_l | R_r> for nl left and nr right vectors (complex dots);
// result in device memory out[l * nr + r] (double2).
// out[l * out_ld + r]; out_ld = 0 means nr.
void block_dots(kgf_ctx* ctx, const double2* Lv, int64_t l_col, int nl,
                const double2* Rv, int64_t r_col, int nr, int64_t D, double2* out,
                int64_t out_ld = 0);

// ---- ABI helpers (api.hip) -------------------------------------------------
// Runs f, turning kgf::Error and other exceptions into a return code and the
// thread-local message of kgf_last_error.
// Named host range around a phase of the path, seen by tracers
// (rocprofv3 --marker-trace); a no-op when no tool is attached.  Popped on
// every exit, exceptions included.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

int abi_guard_impl(void* state, void (*call)(void*));
template <class F>
int abi_guard(F&& f) {
    return abi_guard_impl(&f, [](void* p) { (*static_cast<F*>(p))(); });
}
void check_prop_opts(const kgf_prop_opts* o);
// the uniqueness fields of ground-state options are valid
bool gs_unique_opts_ok(const kgf_gs_opts* o);
SilOpts to_sil_opts(const kgf_prop_opts* o);

// One SIL step of every column of every group (reorth 0, single-pass H.v),
// each kernel launched once for all of them.  Results equal those of
// sil_propagate on each group separately (bitwise: same kernels per group).
void sil_step_groups(kgf_ctx* ctx, const std::vector<GroupSpec>& groups, const std::vector<double2*>& psi,
                     const std::vector<int64_t>& ld, const SilOpts& o);
// reserve the workspaces of the largest grouped step a caller will run
// (avoids growing them step by step)
void sil_groups_reserve(kgf_ctx* ctx, const std::vector<GroupSpec>& groups, int m);

// ---- greens (greens.hip) -------------------------------------------------
void greens_eq(kgf_ctx* ctx, kgf_model* model, const kgf_sector* sec, const double2* psi0,
               double E0, const int32_t* orbs, int norb, int nt, int spg, const SilOpts& o,
               int batch, double2* Gg_host, double2* Gl_host);

}  // namespace kgf
