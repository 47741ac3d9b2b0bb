// C ABI of libkgf: handles, argument checking, error plumbing, workspace
// and kernel timing.  The numerical work lives in basis.hip,
// hamiltonian.hip, krylov.hip and greens.hip.
#include <array>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "kgf_internal.h"

namespace {
thread_local std::string g_last_error;

// Device scratch of kgf_propagate_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes the symbol itself to a kernel; it
// uses the device address resolved per device at kgf_create.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::array<void*, kMaxDevices> g_scratch_addr{};
std::mutex g_scratch_mu;

// with `device` current
void resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device]) return;
    void* p = nullptr;
    KGF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    KGF_REQUIRE(p != nullptr, KGF_EHIP, "kgf_create: no device address for the no-allocation scratch");
    g_scratch_addr[device] = p;
}
}

namespace kgf {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

DevBuf::~DevBuf() {
    if (p) (void)hipFree(p);
}

void DevBuf::reserve(size_t n) {
    if (n <= bytes && p) return;
    if (p) {
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(KGF_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
}

void* workspace(kgf_ctx* ctx, const std::string& name, size_t bytes) {
    auto& slot = ctx->ws[name];
    if (!slot) slot.reset(new DevBuf());
    slot->reserve(bytes < 256 ? 256 : bytes);
    return slot->p;
}

void release_ws(kgf_ctx* ctx, const char* name) {
    auto it = ctx->ws.find(name);
    if (it != ctx->ws.end()) {
        sync(ctx);
        ctx->ws.erase(it);
    }
}

void* host_scratch(kgf_ctx* ctx, size_t bytes) {
    if (bytes > ctx->host_scratch_bytes) {
        if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
        ctx->host_scratch = nullptr;
        KGF_HIP(hipHostMalloc(&ctx->host_scratch, bytes, hipHostMallocDefault));
        ctx->host_scratch_bytes = bytes;
    }
    return ctx->host_scratch;
}

void sync(kgf_ctx* ctx) { KGF_HIP(hipStreamSynchronize(ctx->stream)); }

void* upload_table(kgf_ctx* ctx, const std::string& name, const void* host, size_t n) {
    auto it = ctx->ws.find(name);
    if (it == ctx->ws.end() || !it->second || it->second->bytes < n) sync(ctx);   // growing frees the old buffer
    void* dev = workspace(ctx, name, n);
    const int i = ctx->stage_next;
    ctx->stage_next = (i + 1) % kgf_ctx::kStageSlots;
    if (ctx->stage_ev[i]) KGF_HIP(hipEventSynchronize(ctx->stage_ev[i]));   // the slot's previous copy is done
    if (ctx->stage_bytes[i] < n) {
        if (ctx->stage[i]) KGF_HIP(hipHostFree(ctx->stage[i]));
        ctx->stage[i] = nullptr;
        KGF_HIP(hipHostMalloc(&ctx->stage[i], n, hipHostMallocDefault));
        ctx->stage_bytes[i] = n;
    }
    std::memcpy(ctx->stage[i], host, n);
    KGF_HIP(hipMemcpyAsync(dev, ctx->stage[i], n, hipMemcpyHostToDevice, ctx->stream));
    if (!ctx->stage_ev[i]) KGF_HIP(hipEventCreateWithFlags(&ctx->stage_ev[i], hipEventDisableTiming));
    KGF_HIP(hipEventRecord(ctx->stage_ev[i], ctx->stream));
    return dev;
}

uint64_t next_version() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

void drop_graphs(kgf_ctx* ctx) {
    if (ctx->sil_graphs.empty()) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& g : ctx->sil_graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    ctx->sil_graphs.clear();
}

void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(KGF_EHIP, std::string("launch of ") + what + ": " + hipGetErrorString(e));
}

void ensure_device_fits(size_t bytes, const char* what) {
    size_t free_b = 0, total_b = 0;
    KGF_HIP(hipMemGetInfo(&free_b, &total_b));
    if (bytes > free_b)
        fail(KGF_ENOMEM, std::string(what) + ": needs " + std::to_string(bytes >> 20) +
                             " MiB, " + std::to_string(free_b >> 20) + " MiB free");
}

void progress(kgf_ctx* ctx, const char* phase, int64_t done, int64_t total) {
    if (!ctx->progress) return;
    sync(ctx);
    ctx->progress(ctx->progress_user, phase, done, total);
}

static hipEvent_t take_event(kgf_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    KGF_HIP(hipEventCreate(&e));
    return e;
}

Prof::Prof(kgf_ctx* c, const char* n, double by) : ctx(c), name(n), bytes(by) {
    if (!ctx->prof_on) return;
    auto& st = ctx->prof[name];
    bool take = (st.launches % ctx->prof_every) == 0;
    st.launches++;
    if (!take) return;
    a = take_event(ctx);
    b = take_event(ctx);
    KGF_HIP(hipEventRecord(a, ctx->stream));
}

Prof::~Prof() {
    if (!a) return;
    if (hipEventRecord(b, ctx->stream) == hipSuccess)
        ctx->pending.push_back({name, a, b, bytes});
}

}  // namespace kgf

using namespace kgf;

template <class F>
static int guarded(F&& f) {
    try {
        f();
        return KGF_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return KGF_EHIP;
    } catch (...) {
        g_last_error = "unknown error";
        return KGF_EHIP;
    }
}

namespace kgf {
int abi_guard_impl(void* state, void (*call)(void*)) {
    return guarded([&] { call(state); });
}
}  // namespace kgf

static bool finite_all(const double* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

namespace kgf {
void check_prop_opts(const kgf_prop_opts* o) {
    KGF_REQUIRE(o, KGF_EINVAL, "propagation options are NULL");
    KGF_REQUIRE(o->krylov_dim >= 1 && o->krylov_dim <= kMaxKrylov, KGF_EUNSUPPORTED,
                "krylov_dim must be in 1..128");
    KGF_REQUIRE(o->reorth >= 0 && o->reorth <= 2, KGF_EINVAL, "reorth must be 0, 1 or 2");
    KGF_REQUIRE(o->direction >= -1 && o->direction <= 1, KGF_EINVAL, "direction must be -1, 0 or 1");
    KGF_REQUIRE(std::isfinite(o->dt) && std::isfinite(o->shift) && std::isfinite(o->breakdown_tol) &&
                    o->breakdown_tol >= 0.0,
                KGF_EINVAL, "non-finite propagation option");
}

bool gs_unique_opts_ok(const kgf_gs_opts* o) {
    return (o->unique_check == 0 || o->unique_check == 1) && std::isfinite(o->unique_tol) && o->unique_tol >= 0.0 &&
           o->unique_tol < 1.0;
}

SilOpts to_sil_opts(const kgf_prop_opts* o) {
    SilOpts s;
    s.m = o->krylov_dim;
    s.reorth = o->reorth;
    s.dt = o->dt;
    s.direction = o->direction;
    s.shift = o->shift;
    s.breakdown_tol = o->breakdown_tol;
    return s;
}
}  // namespace kgf

extern "C" {

const char* kgf_last_error(void) { return g_last_error.c_str(); }
int kgf_version(void) { return KGF_ABI_VERSION; }

int kgf_create(kgf_ctx** out, int hip_device, void* hip_stream) {
    return guarded([&] {
        KGF_REQUIRE(out, KGF_EINVAL, "kgf_create: out is NULL");
        int ndev = 0;
        KGF_HIP(hipGetDeviceCount(&ndev));
        KGF_REQUIRE(hip_device >= 0 && hip_device < ndev, KGF_EINVAL,
                    "kgf_create: device " + std::to_string(hip_device) + " out of range");
        KGF_REQUIRE(hip_device < kMaxDevices, KGF_EUNSUPPORTED, "kgf_create: device index above 63");
        KGF_HIP(hipSetDevice(hip_device));
        resolve_scratch(hip_device);
        std::unique_ptr<kgf_ctx> c(new kgf_ctx());
        c->device = hip_device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        build_binomials(c.get());
        *out = c.release();
    });
}

void kgf_destroy(kgf_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
    drop_graphs(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (int i = 0; i < kgf_ctx::kStageSlots; ++i) {
        if (ctx->stage_ev[i]) (void)hipEventDestroy(ctx->stage_ev[i]);
        if (ctx->stage[i]) (void)hipHostFree(ctx->stage[i]);
    }
    delete ctx;
}

int kgf_set_stream(kgf_ctx* ctx, void* hip_stream) {
    return guarded([&] {
        KGF_REQUIRE(ctx, KGF_EINVAL, "kgf_set_stream: ctx is NULL");
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    });
}

int kgf_model_create(kgf_ctx* ctx, const kgf_model_desc* d, kgf_model** out) {
    return guarded([&] {
        KGF_REQUIRE(ctx && d && out, KGF_EINVAL, "kgf_model_create: NULL argument");
        KGF_REQUIRE(d->L >= 1 && d->L <= kMaxL, KGF_EUNSUPPORTED,
                    "kgf_model_create: L must be in 1.." + std::to_string(kMaxL));
        KGF_REQUIRE(d->n_bonds >= 0 && d->n_bonds <= kMaxBonds, KGF_EUNSUPPORTED,
                    "kgf_model_create: n_bonds must be in 0..127");
        KGF_REQUIRE(d->eps_up && d->eps_dn && d->U, KGF_EINVAL,
                    "kgf_model_create: eps_up, eps_dn and U are required");
        KGF_REQUIRE(d->n_bonds == 0 || (d->bond_i && d->bond_j && d->t_bond), KGF_EINVAL,
                    "kgf_model_create: bond arrays are required");
        std::unique_ptr<kgf_model> m(new kgf_model());
        m->ctx = ctx;
        m->L = d->L;
        m->nb = d->n_bonds;
        for (int b = 0; b < d->n_bonds; ++b) {
            int i = d->bond_i[b], j = d->bond_j[b];
            KGF_REQUIRE(i >= 0 && i < d->L && j >= 0 && j < d->L && i != j, KGF_EINVAL,
                        "kgf_model_create: bond " + std::to_string(b) + " has bad sites");
            m->bi.push_back(i);
            m->bj.push_back(j);
            m->t.push_back(d->t_bond[b]);
        }
        m->eps_up.assign(d->eps_up, d->eps_up + d->L);
        m->eps_dn.assign(d->eps_dn, d->eps_dn + d->L);
        m->U.assign(d->U, d->U + d->L);
        KGF_REQUIRE(finite_all(m->t.data(), m->nb) && finite_all(d->eps_up, d->L) &&
                        finite_all(d->eps_dn, d->L) && finite_all(d->U, d->L),
                    KGF_EINVAL, "kgf_model_create: non-finite parameter");
        KGF_HIP(hipSetDevice(ctx->device));
        upload_params(m.get());
        m->version = next_version();
        *out = m.release();
    });
}

int kgf_model_set_params(kgf_model* m, const kgf_model_desc* d) {
    return guarded([&] {
        KGF_REQUIRE(m && d, KGF_EINVAL, "kgf_model_set_params: NULL argument");
        KGF_REQUIRE(d->L == m->L && d->n_bonds == m->nb, KGF_EINVAL,
                    "kgf_model_set_params: L and the number of bonds must stay the same");
        KGF_REQUIRE(d->eps_up && d->eps_dn && d->U && (m->nb == 0 || (d->bond_i && d->bond_j && d->t_bond)),
                    KGF_EINVAL, "kgf_model_set_params: NULL parameter array");
        for (int b = 0; b < m->nb; ++b)
            KGF_REQUIRE(d->bond_i[b] == m->bi[b] && d->bond_j[b] == m->bj[b], KGF_EINVAL,
                        "kgf_model_set_params: bond " + std::to_string(b) + " differs");
        KGF_REQUIRE(finite_all(d->t_bond, m->nb) && finite_all(d->eps_up, m->L) && finite_all(d->eps_dn, m->L) &&
                        finite_all(d->U, m->L),
                    KGF_EINVAL, "kgf_model_set_params: non-finite parameter");
        model_set_params(m, d->t_bond, d->eps_up, d->eps_dn, d->U);
    });
}

int kgf_model_get_params(const kgf_model* m, double* host_t, double* host_eps_up, double* host_eps_dn,
                         double* host_U) {
    return guarded([&] {
        KGF_REQUIRE(m, KGF_EINVAL, "kgf_model_get_params: NULL model");
        if (host_t) std::copy(m->t.begin(), m->t.end(), host_t);
        if (host_eps_up) std::copy(m->eps_up.begin(), m->eps_up.end(), host_eps_up);
        if (host_eps_dn) std::copy(m->eps_dn.begin(), m->eps_dn.end(), host_eps_dn);
        if (host_U) std::copy(m->U.begin(), m->U.end(), host_U);
    });
}

void kgf_model_destroy(kgf_model* m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream);
    delete m;
}

int kgf_sector_create(kgf_ctx* ctx, int L, int n_up, int n_dn, kgf_sector** out) {
    return guarded([&] {
        KGF_REQUIRE(ctx && out, KGF_EINVAL, "kgf_sector_create: NULL argument");
        KGF_REQUIRE(L >= 1 && L <= kMaxL, KGF_EUNSUPPORTED, "kgf_sector_create: L out of range");
        KGF_REQUIRE(n_up >= 0 && n_up <= L && n_dn >= 0 && n_dn <= L, KGF_EINVAL,
                    "kgf_sector_create: particle numbers out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        std::unique_ptr<kgf_sector> s(new kgf_sector());
        s->ctx = ctx;
        s->L = L;
        s->n_up = n_up;
        s->n_dn = n_dn;
        s->d_up = binom_host(L, n_up);
        s->d_dn = binom_host(L, n_dn);
        s->masks_up.reserve(sizeof(uint32_t) * s->d_up);
        s->masks_dn.reserve(sizeof(uint32_t) * s->d_dn);
        build_masks(ctx, L, n_up, s->masks_up.as<uint32_t>(), s->d_up);
        build_masks(ctx, L, n_dn, s->masks_dn.as<uint32_t>(), s->d_dn);
        sync(ctx);
        *out = s.release();
    });
}

void kgf_sector_destroy(kgf_sector* s) {
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    delete s;
}

int kgf_sector_dims(const kgf_sector* s, int64_t* d_up, int64_t* d_dn) {
    return guarded([&] {
        KGF_REQUIRE(s && d_up && d_dn, KGF_EINVAL, "kgf_sector_dims: NULL argument");
        *d_up = s->d_up;
        *d_dn = s->d_dn;
    });
}

int kgf_sector_states(kgf_ctx* ctx, const kgf_sector* s, int spin, uint32_t* host_masks) {
    return guarded([&] {
        KGF_REQUIRE(ctx && s && host_masks, KGF_EINVAL, "kgf_sector_states: NULL argument");
        KGF_REQUIRE(spin == 0 || spin == 1, KGF_EINVAL, "kgf_sector_states: spin must be 0 or 1");
        KGF_HIP(hipSetDevice(ctx->device));
        const DevBuf& b = spin == 0 ? s->masks_up : s->masks_dn;
        int64_t D = spin == 0 ? s->d_up : s->d_dn;
        if (D == 0) return;
        KGF_HIP(hipMemcpyAsync(host_masks, b.p, sizeof(uint32_t) * D, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    });
}

int kgf_sector_rank(kgf_ctx* ctx, const kgf_sector* s, int spin, const uint32_t* masks,
                    int64_t n, int64_t* ranks) {
    return guarded([&] {
        KGF_REQUIRE(ctx && s, KGF_EINVAL, "kgf_sector_rank: NULL argument");
        KGF_REQUIRE(spin == 0 || spin == 1, KGF_EINVAL, "kgf_sector_rank: spin must be 0 or 1");
        KGF_REQUIRE(n >= 0 && (n == 0 || (masks && ranks)), KGF_EINVAL, "kgf_sector_rank: bad buffers");
        KGF_HIP(hipSetDevice(ctx->device));
        if (n) rank_masks(ctx, masks, n, spin == 0 ? s->n_up : s->n_dn, ranks);
    });
}

int kgf_hop_table(kgf_ctx* ctx, const kgf_model* model, int n, int32_t* host_count,
                  uint32_t* host_entries, int* host_width) {
    return guarded([&] {
        KGF_REQUIRE(ctx && model && host_width, KGF_EINVAL, "kgf_hop_table: NULL argument");
        KGF_REQUIRE(n >= 0 && n <= model->L, KGF_EINVAL, "kgf_hop_table: n out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        HopTable& t = hop_table(const_cast<kgf_model*>(model), n);
        *host_width = t.width;
        if (t.D == 0) return;
        if (host_count)
            KGF_HIP(hipMemcpyAsync(host_count, t.count.p, sizeof(int32_t) * t.D,
                                   hipMemcpyDeviceToHost, ctx->stream));
        if (host_entries && t.width)
            KGF_HIP(hipMemcpyAsync(host_entries, t.ent.p, sizeof(uint32_t) * t.D * t.width,
                                   hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    });
}

int kgf_apply_h(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* s, const kgf_c128* v,
                kgf_c128* w, int nvec, int64_t ld) {
    return guarded([&] {
        KGF_REQUIRE(ctx && model && s, KGF_EINVAL, "kgf_apply_h: NULL handle");
        KGF_REQUIRE(model->L == s->L, KGF_EINVAL, "kgf_apply_h: model and sector L differ");
        KGF_REQUIRE(nvec >= 0 && ld >= s->dim(), KGF_EINVAL, "kgf_apply_h: bad nvec / ld");
        if (nvec == 0 || s->dim() == 0) return;
        KGF_REQUIRE(v && w, KGF_EINVAL, "kgf_apply_h: NULL vector");
        KGF_HIP(hipSetDevice(ctx->device));
        apply_h(ctx, const_cast<kgf_model*>(model), s, reinterpret_cast<const double2*>(v),
                reinterpret_cast<double2*>(w), nvec, ld);
    });
}

int kgf_apply_c(kgf_ctx* ctx, const kgf_sector* src, const kgf_sector* dst, int orbital,
                int dagger, const kgf_c128* v, kgf_c128* w, int nvec, int64_t ld_src,
                int64_t ld_dst) {
    return guarded([&] {
        KGF_REQUIRE(ctx && src && dst, KGF_EINVAL, "kgf_apply_c: NULL handle");
        KGF_REQUIRE(src->L == dst->L, KGF_EINVAL, "kgf_apply_c: sectors of different L");
        int site = orbital >> 1, spin = orbital & 1;
        KGF_REQUIRE(orbital >= 0 && site < src->L, KGF_EINVAL, "kgf_apply_c: orbital out of range");
        int du = spin == 0 ? (dagger ? 1 : -1) : 0;
        int dd = spin == 1 ? (dagger ? 1 : -1) : 0;
        KGF_REQUIRE(dst->n_up == src->n_up + du && dst->n_dn == src->n_dn + dd, KGF_EINVAL,
                    "kgf_apply_c: dst is not the sector reached by the operator");
        KGF_REQUIRE(nvec >= 0 && ld_src >= src->dim() && ld_dst >= dst->dim(), KGF_EINVAL,
                    "kgf_apply_c: bad nvec / ld");
        if (nvec == 0 || dst->dim() == 0) return;
        KGF_REQUIRE(w && (v || src->dim() == 0), KGF_EINVAL, "kgf_apply_c: NULL vector");
        KGF_HIP(hipSetDevice(ctx->device));
        apply_c(ctx, src, dst, orbital, dagger, reinterpret_cast<const double2*>(v),
                reinterpret_cast<double2*>(w), nvec, ld_src, ld_dst);
    });
}


// largest of n device doubles (n small: the per-column error estimates)
static double host_max(kgf_ctx* ctx, const double* dev, int n) {
    std::vector<double> h((size_t)n);
    KGF_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    double m = 0.0;
    for (double v : h) m = std::fmax(m, v);
    return m;
}

int kgf_propagate(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* s, kgf_c128* psi,
                  int nvec, int64_t ld, int nsteps, const kgf_prop_opts* opts, double* host_err_est,
                  double* host_norm_drift) {
    return guarded([&] {
        KGF_REQUIRE(ctx && model && s, KGF_EINVAL, "kgf_propagate: NULL handle");
        KGF_REQUIRE(model->L == s->L, KGF_EINVAL, "kgf_propagate: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(nvec >= 0 && nsteps >= 0 && ld >= s->dim(), KGF_EINVAL,
                    "kgf_propagate: bad nvec / nsteps / ld");
        if (host_err_est) *host_err_est = 0.0;
        if (host_norm_drift) *host_norm_drift = 0.0;
        if (nvec == 0 || nsteps == 0 || s->dim() == 0) return;
        KGF_REQUIRE(psi, KGF_EINVAL, "kgf_propagate: NULL psi");
        KGF_HIP(hipSetDevice(ctx->device));
        double* err = host_err_est ? static_cast<double*>(workspace(ctx, "sil_err", sizeof(double) * nvec)) : nullptr;
        double* drift =
            host_norm_drift ? static_cast<double*>(workspace(ctx, "sil_drift", sizeof(double) * nvec)) : nullptr;
        sil_propagate(ctx, const_cast<kgf_model*>(model), s, reinterpret_cast<double2*>(psi), nvec,
                      ld, nsteps, to_sil_opts(opts), err, drift);
        if (host_err_est) *host_err_est = host_max(ctx, err, nvec);
        if (host_norm_drift) *host_norm_drift = host_max(ctx, drift, nvec);
    });
}

int kgf_propagate_noalloc(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* s, kgf_c128* psi,
                          int nvec, int64_t ld, int nsteps, const kgf_prop_opts* opts, double* host_err_est) {
    return guarded([&] {
        KGF_REQUIRE(ctx && model && s, KGF_EINVAL, "kgf_propagate_noalloc: NULL handle");
        KGF_REQUIRE(model->L == s->L, KGF_EINVAL, "kgf_propagate_noalloc: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(nvec >= 0 && nvec <= 65535 && nsteps >= 0 && ld >= s->dim(), KGF_EINVAL,
                    "kgf_propagate_noalloc: bad nvec / nsteps / ld");
        if (host_err_est) *host_err_est = 0.0;
        if (nvec == 0 || nsteps == 0 || s->dim() == 0) return;
        KGF_REQUIRE(psi, KGF_EINVAL, "kgf_propagate_noalloc: NULL psi");
        KGF_REQUIRE(hop_table_ready(model, s->n_up) && hop_table_ready(model, s->n_dn), KGF_EINVAL,
                    "kgf_propagate_noalloc: the model's hopping tables for this sector are not built yet "
                    "(one kgf_apply_h or kgf_propagate on the sector builds them)");
        const size_t need = sil_scratch_bytes(ctx, s, nvec, opts->krylov_dim, opts->reorth);
        KGF_REQUIRE(need <= kNoAllocScratchBytes, KGF_EUNSUPPORTED,
                    "kgf_propagate_noalloc: needs " + std::to_string((need + (1 << 20) - 1) >> 20) +
                        " MiB of scratch (krylov_dim x nvec x D complex128 plus scalars); the limit is " +
                        std::to_string(kNoAllocScratchBytes >> 20) + " MiB");
        KGF_HIP(hipSetDevice(ctx->device));
        void* base = g_scratch_addr[ctx->device];
        KGF_REQUIRE(base != nullptr, KGF_EHIP, "kgf_propagate_noalloc: scratch address not resolved");
        double* err = sil_propagate_in(ctx, const_cast<kgf_model*>(model), s, reinterpret_cast<double2*>(psi), nvec,
                                       ld, nsteps, to_sil_opts(opts), base, host_err_est != nullptr);
        if (host_err_est) {   // a fixed-size host copy: no allocation on either side
            double h[64];
            double mx = 0.0;
            for (int c0 = 0; c0 < nvec; c0 += 64) {
                const int n = std::min(64, nvec - c0);
                KGF_HIP(hipMemcpyAsync(h, err + c0, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
                sync(ctx);
                for (int i = 0; i < n; ++i) mx = std::fmax(mx, h[i]);
            }
            *host_err_est = mx;
        }
    });
}

int kgf_ground_state(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* s,
                     const kgf_gs_opts* o, const kgf_c128* v0, kgf_c128* psi0, double* host_E0,
                     kgf_gs_info* info) {
    int conv_code = KGF_OK;
    int rc = guarded([&] {
        KGF_REQUIRE(ctx && model && s && o && host_E0, KGF_EINVAL, "kgf_ground_state: NULL argument");
        KGF_REQUIRE(model->L == s->L, KGF_EINVAL, "kgf_ground_state: model and sector L differ");
        KGF_REQUIRE(s->dim() > 0, KGF_EINVAL, "kgf_ground_state: empty sector");
        KGF_REQUIRE(v0 && psi0, KGF_EINVAL, "kgf_ground_state: NULL vector");
        KGF_REQUIRE(o->max_iter >= 1 && o->max_iter <= 4000 && o->check_every >= 1 &&
                        std::isfinite(o->tol) && o->tol >= 0.0 && o->reorth >= 0 && o->reorth <= 2 &&
                        (o->unique_check == 0 || o->unique_check == 1) && std::isfinite(o->unique_tol) &&
                        o->unique_tol >= 0.0 && o->unique_tol < 1.0,
                    KGF_EINVAL, "kgf_ground_state: bad options");
        KGF_HIP(hipSetDevice(ctx->device));
        GsResult r = ground_state(ctx, const_cast<kgf_model*>(model), s,
                                  reinterpret_cast<const double2*>(v0),
                                  reinterpret_cast<double2*>(psi0), o->tol, o->max_iter,
                                  o->check_every, o->reorth);
        *host_E0 = r.E0;
        double f2 = -1.0;
        if (o->unique_check && r.converged)
            f2 = gs_fidelity2(ctx, const_cast<kgf_model*>(model), s, reinterpret_cast<const double2*>(psi0), o);
        if (info) {
            info->iters = r.iters;
            info->converged = r.converged ? 1 : 0;
            info->residual = r.residual;
            info->fidelity2 = f2;
        }
        if (!r.converged) {
            g_last_error = "ground-state Lanczos did not converge within max_iter";
            conv_code = KGF_ENOCONV;
        } else if (o->unique_check && !(f2 >= 1.0 - (o->unique_tol > 0.0 ? o->unique_tol : 1e-10))) {
            g_last_error = "the ground state is not unique: two Lanczos starts give |<0_a|0_b>|^2 = " + std::to_string(f2);
            conv_code = KGF_EDEGENERATE;
        }
    });
    return rc != KGF_OK ? rc : conv_code;
}

int kgf_greens_eq(kgf_ctx* ctx, const kgf_model* model, const kgf_sector* s, const kgf_c128* psi0,
                  double E0, const int32_t* host_orbs, int n_orb, int nt, int steps_per_grid,
                  const kgf_prop_opts* opts, int batch, kgf_c128* host_G_greater,
                  kgf_c128* host_G_lesser) {
    return guarded([&] {
        KGF_REQUIRE(ctx && model && s && psi0 && host_orbs, KGF_EINVAL, "kgf_greens_eq: NULL argument");
        KGF_REQUIRE(model->L == s->L, KGF_EINVAL, "kgf_greens_eq: model and sector L differ");
        check_prop_opts(opts);
        KGF_REQUIRE(n_orb >= 1 && nt >= 1 && steps_per_grid >= 1 && batch >= 0 && std::isfinite(E0),
                    KGF_EINVAL, "kgf_greens_eq: bad sizes");
        for (int a = 0; a < n_orb; ++a)
            KGF_REQUIRE(host_orbs[a] >= 0 && (host_orbs[a] >> 1) < s->L, KGF_EINVAL,
                        "kgf_greens_eq: orbital out of range");
        KGF_HIP(hipSetDevice(ctx->device));
        greens_eq(ctx, const_cast<kgf_model*>(model), s, reinterpret_cast<const double2*>(psi0), E0,
                  host_orbs, n_orb, nt, steps_per_grid, to_sil_opts(opts), batch,
                  reinterpret_cast<double2*>(host_G_greater), reinterpret_cast<double2*>(host_G_lesser));
    });
}

int kgf_set_progress(kgf_ctx* ctx, kgf_progress_fn fn, void* user) {
    return guarded([&] {
        KGF_REQUIRE(ctx, KGF_EINVAL, "kgf_set_progress: ctx is NULL");
        ctx->progress = fn;
        ctx->progress_user = user;
    });
}

int kgf_set_option(kgf_ctx* ctx, int option, int value) {
    return guarded([&] {
        KGF_REQUIRE(ctx, KGF_EINVAL, "kgf_set_option: ctx is NULL");
        drop_graphs(ctx);   // captured steps follow the kernel choices in force when captured
        if (option == KGF_OPT_HV_PASSES) {
            KGF_REQUIRE(value >= 0 && value <= 4, KGF_EINVAL, "kgf_set_option: HV_PASSES must be 0..4");
            ctx->hv_passes = value;
        } else if (option == KGF_OPT_HV_STRIP) {
            KGF_REQUIRE(value == 0 || value == 8 || value == 16 || value == 32 || value == 64 || value == 128,
                        KGF_EINVAL, "kgf_set_option: HV_STRIP must be 0, 8, 16, 32, 64 or 128");
            ctx->hv_strip = value;
        } else if (option == KGF_OPT_GS_MAX_BASIS) {
            KGF_REQUIRE(value == 0 || value >= 8, KGF_EINVAL, "kgf_set_option: GS_MAX_BASIS must be 0 or >= 8");
            ctx->gs_max_basis = value;
        } else if (option == KGF_OPT_PHI_EVERY) {
            KGF_REQUIRE(value >= 0, KGF_EINVAL, "kgf_set_option: PHI_EVERY must be >= 0");
            ctx->phi_every = value;
        } else if (option == KGF_OPT_ADJ_EVERY) {
            KGF_REQUIRE(value >= 0, KGF_EINVAL, "kgf_set_option: ADJ_EVERY must be >= 0");
            ctx->adj_every = value;
        } else if (option == KGF_OPT_HV_TUNE) {
            KGF_REQUIRE(value == 0 || value == 1, KGF_EINVAL, "kgf_set_option: HV_TUNE must be 0 or 1");
            ctx->hv_tune = value;
        } else if (option == KGF_OPT_CG_MAX_ITER) {
            KGF_REQUIRE(value >= 0, KGF_EINVAL, "kgf_set_option: CG_MAX_ITER must be >= 0");
            ctx->cg_max_iter = value;
        } else if (option == KGF_OPT_LOCKSTEP) {
            KGF_REQUIRE(value == 0 || value == 1, KGF_EINVAL, "kgf_set_option: LOCKSTEP must be 0 or 1");
            ctx->lockstep = value;
        } else if (option == KGF_OPT_GRAPHS) {
            KGF_REQUIRE(value == 0 || value == 1, KGF_EINVAL, "kgf_set_option: GRAPHS must be 0 or 1");
            ctx->use_graphs = value;
        } else if (option == KGF_OPT_HV_FUSE) {
            KGF_REQUIRE(value == 0 || value == 1, KGF_EINVAL, "kgf_set_option: HV_FUSE must be 0 or 1");
            ctx->hv_fuse = value;
        } else if (option == KGF_OPT_HV_SEG) {
            KGF_REQUIRE(value == 0 || value == 1, KGF_EINVAL, "kgf_set_option: HV_SEG must be 0 or 1");
            ctx->hv_seg = value;
        } else if (option == KGF_OPT_HV_UP_THREADS) {
            KGF_REQUIRE(value == 256 || value == 512 || value == 1024, KGF_EINVAL,
                        "kgf_set_option: HV_UP_THREADS must be 256, 512 or 1024");
            ctx->hv_up_threads = value;
        } else {
            fail(KGF_EINVAL, "kgf_set_option: unknown option");
        }
    });
}

int kgf_profile_begin(kgf_ctx* ctx, int sample_every) {
    return guarded([&] {
        KGF_REQUIRE(ctx && sample_every >= 1, KGF_EINVAL, "kgf_profile_begin: bad argument");
        ctx->prof.clear();
        ctx->prof_on = true;
        ctx->prof_every = sample_every;
    });
}

int kgf_profile_end(kgf_ctx* ctx, kgf_kernel_stat* out, int max_classes) {
    int n = 0;
    int rc = guarded([&] {
        KGF_REQUIRE(ctx && (out || max_classes == 0), KGF_EINVAL, "kgf_profile_end: bad argument");
        KGF_HIP(hipSetDevice(ctx->device));
        sync(ctx);
        for (auto& p : ctx->pending) {
            float ms = 0.f;
            KGF_HIP(hipEventElapsedTime(&ms, p.a, p.b));
            auto& st = ctx->prof[p.name];
            st.sampled++;
            st.ms += ms;
            st.bytes += p.bytes;
            ctx->event_pool.push_back(p.a);
            ctx->event_pool.push_back(p.b);
        }
        ctx->pending.clear();
        ctx->prof_on = false;
        for (auto& kv : ctx->prof) {
            if (n >= max_classes) break;
            std::memset(out[n].name, 0, sizeof(out[n].name));
            std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
            out[n].launches = kv.second.launches;
            out[n].sampled = kv.second.sampled;
            out[n].sampled_ms = kv.second.ms;
            out[n].sampled_bytes = kv.second.bytes;
            ++n;
        }
    });
    return rc != KGF_OK ? rc : n;
}

}  // extern "C"
