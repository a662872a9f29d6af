// C ABI entry points of libgs: plan construction ("init" of the paper's
// Freq2Wave, Sec. 6.2), applies of T and T^H, plan queries and the host-only
// basis queries.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <stdexcept>
#include <thread>
#include <vector>

#include "common.hpp"
#include "host_math.hpp"
#include "prof.hpp"

#include <mutex>

namespace gs {
size_t adjoint_part_elems(int dim, int64_t M, int nb, int ng);
hipError_t device_point_tables(Plan& P, const double* xi_host, const double* mu_host, hipStream_t s);
}

namespace {

thread_local char g_hip_msg[256] = "";

int hip_fail(hipError_t e) {
    std::snprintf(g_hip_msg, sizeof g_hip_msg, "HIP error %d: %s", (int)e, hipGetErrorString(e));
    return GS_ERR_HIP;
}

template <class P>
hipError_t dalloc(gs::Plan& pl, P*& ptr, size_t elems) {
    ptr = nullptr;
    if (elems == 0) return hipSuccess;
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, elems * sizeof(P));
    if (e != hipSuccess) return e;
    ptr = static_cast<P*>(v);
    pl.bytes += (int64_t)(elems * sizeof(P));
    return hipSuccess;
}

template <class P>
void dfree(P*& ptr) {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
}

template <class T>
void free_prec(gs::PrecData<T>& d) {
    dfree(d.pos); dfree(d.chx); dfree(d.chy); dfree(d.smu); dfree(d.win); dfree(d.deap); dfree(d.tw);
    dfree(d.grid); dfree(d.sr); dfree(d.sc); dfree(d.part); dfree(d.vbuf); dfree(d.ybuf);
    d.present = false;
}

void free_plan(gs::Plan& P) {
    free_prec(P.d64);
    free_prec(P.d32);
    dfree(P.perm); dfree(P.cell_start); dfree(P.tile_order);
    dfree(P.smu64); dfree(P.b); dfree(P.r); dfree(P.q); dfree(P.ps); dfree(P.ss);
    dfree(P.q32); dfree(P.r32); dfree(P.p32); dfree(P.s32); dfree(P.xbest);
    dfree(P.red); dfree(P.scal); dfree(P.hist);
    if (P.host_scal) (void)hipHostFree(P.host_scal);
    P.host_scal = nullptr;
    if (P.ev_fork) (void)hipEventDestroy(P.ev_fork);
    if (P.ev_join) (void)hipEventDestroy(P.ev_join);
    if (P.side) (void)hipStreamDestroy(P.side);
    P.ev_fork = P.ev_join = nullptr;
    P.side = nullptr;
}

int hw_threads() {
    unsigned n = std::thread::hardware_concurrency();
    return n == 0 ? 4 : (int)std::min(n, 64u);
}

// Smallest a in 0..3 such that every value times 2^a is an integer (all
// frequencies lie on the grid 2^-a Z), or -1.
int uniform_level(const double* v, int64_t n) {
    int a = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(std::fabs(v[i]) < 0x1p50)) return -1;
        while (a <= 3 && std::ldexp(v[i], a) != std::floor(std::ldexp(v[i], a))) ++a;
        if (a > 3) return -1;
    }
    return a;
}


template <class T>
hipError_t upload_prec(gs::Plan& P, int w, int deg, double beta) {
    using namespace gs;
    PrecData<T>& d = prec<T>(P);
    const size_t M = P.M;
    d.present = true;
    d.w = w;
    d.deg = deg;
    // window and deapodization.  On exact nodes (P.exact) the window is the
    // linear hat, which at a node has the taps (.., 0, 1, 0, ..): interpolation
    // and spreading then read and write the node itself, with no window error,
    // and no deapodization is needed.
    const KBWindow kb = make_window(w, deg, beta);
    {
        std::vector<T> hw(kb.coef.begin(), kb.coef.end());
        if (P.exact) {
            std::fill(hw.begin(), hw.end(), T(0));
            const int j0 = w / 2 - 1, n = deg + 1;   // taps at distance t and t - 1
            hw[j0 * n] = T(0.5); hw[j0 * n + 1] = T(-0.5);
            hw[(j0 + 1) * n] = T(0.5); hw[(j0 + 1) * n + 1] = T(0.5);
        }
        GS_HIP_TRY(dalloc(P, d.win, hw.size()));
        GS_HIP_TRY(hipMemcpy(d.win, hw.data(), hw.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    {
        GS_HIP_TRY(dalloc(P, d.deap, (size_t)P.N));
        std::vector<T> hd(P.N);
        for (int j = 0; j < P.N; ++j) {
            const bool interior = j >= P.nb && j < P.N - P.nb;
            hd[j] = !interior ? T(0) : P.exact ? T(1) : (T)(1.0 / kb.ft((double)(j - P.N / 2) / P.ng));
        }
        GS_HIP_TRY(hipMemcpy(d.deap, hd.data(), hd.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    {
        GS_HIP_TRY(dalloc(P, d.tw, (size_t)P.ng));
        std::vector<cx<T>> ht(P.ng);
        for (int k = 0; k < P.ng; ++k) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / P.ng;
            ht[k] = mk<T>((T)std::cos(a), (T)std::sin(a));
        }
        GS_HIP_TRY(hipMemcpy(d.tw, ht.data(), ht.size() * sizeof(cx<T>), hipMemcpyHostToDevice));
    }
    // workspace
    const size_t gsz = P.dim == 2 ? (size_t)P.ng * P.ng : (size_t)P.ng;
    GS_HIP_TRY(dalloc(P, d.grid, gsz));
    if (P.dim == 2 && P.nb) {
        GS_HIP_TRY(dalloc(P, d.sr, (size_t)2 * P.nb * P.ng));
        GS_HIP_TRY(dalloc(P, d.sc, (size_t)2 * P.nb * P.ng));
    }
    d.part_elems = adjoint_part_elems(P.dim, P.M, P.nb, P.ng);
    GS_HIP_TRY(dalloc(P, d.part, d.part_elems));
    GS_HIP_TRY(dalloc(P, d.vbuf, M));
    GS_HIP_TRY(dalloc(P, d.ybuf, M));
    return hipSuccess;
}

}  // namespace

namespace gs {
hipError_t solver_alloc(Plan& P);

bool g_prof_enabled = false;
thread_local LaunchCtx* g_launch = nullptr;

namespace {
struct ProfRec {
    int id;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;
std::vector<size_t> g_prof_open;
const char* const kKernelNames[K_COUNT] = {
    "fft_rows_T", "fft_cols_T", "fft_sidecols_T", "interp2d", "interp1d", "fft1_T",
    "adj_prep", "boundary_partial", "boundary_final", "spread2d", "side_rows_partial", "side_cols_partial",
    "reduce_strips", "fft_cols_TH", "fft_rows_TH", "fft_sidecols_TH", "spread1d", "fft1_TH", "merge_tiles", "boundary2d", "interp_bnd2d",
    "cnn_first", "cnn_conv32", "cnn_last", "cnn_loss", "cnn_last_bwd", "cnn_conv32_bwd", "cnn_dw32", "cnn_dw_thin",
    "cnn_adam"};

void prof_clear() {
    for (auto& r : g_prof_recs) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    g_prof_recs.clear();
    g_prof_open.clear();
}
}  // namespace

void prof_record(int id, hipStream_t s, bool begin) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        g_prof_recs.push_back({id, e, nullptr});
        g_prof_open.push_back(g_prof_recs.size() - 1);
    } else if (!g_prof_open.empty()) {
        g_prof_recs[g_prof_open.back()].b = e;
        g_prof_open.pop_back();
    } else {
        (void)hipEventDestroy(e);
    }
}
}  // namespace gs

extern "C" {

int gs_version(void) { return GS_VERSION; }

const char* gs_strerror(int code) {
    switch (code) {
        case GS_OK: return "success";
        case GS_NOT_CONVERGED: return "CGLS reached max_iter before the tolerance";
        case GS_ERR_INVALID_ARG: return "invalid argument";
        case GS_ERR_UNSUPPORTED: return "unsupported configuration (p, J or grid size)";
        case GS_ERR_BAD_NODES: return "non-finite frequency or negative/non-finite weight";
        case GS_ERR_NOMEM: return "out of memory";
        case GS_ERR_HIP: return g_hip_msg[0] ? g_hip_msg : "HIP runtime error";
        case GS_ERR_BREAKDOWN: return "CGLS breakdown (||A p||^2 <= 0 or non-finite)";
        case GS_ERR_PRECISION: return "requested precision is not held by this plan";
        case GS_ERR_TOO_LARGE: return "the apply needs more workspace than the static device array holds";
        default: return "unknown status";
    }
}

int gs_plan(gs_plan_t** out, int dim, int J, int p, int64_t M, const double* xi, const double* mu, int precision,
            void* stream) {
    if (!out) return GS_ERR_INVALID_ARG;
    *out = nullptr;
    if (dim != 1 && dim != 2) return GS_ERR_INVALID_ARG;
    if (!xi || M <= 0 || M > (int64_t)std::numeric_limits<int32_t>::max() / 2) return GS_ERR_INVALID_ARG;
    if (precision != GS_F64 && precision != GS_F32 && precision != GS_F32_MIXED) return GS_ERR_INVALID_ARG;
    if (p < 1 || p > 8) return GS_ERR_UNSUPPORTED;
    if (J < 1 || J > (dim == 2 ? 11 : 20)) return GS_ERR_UNSUPPORTED;
    if ((1 << J) < 2 * p) return GS_ERR_UNSUPPORTED;
    // FP32 positions: 32-bit fixed point, log2(grid) bits of cell, >= 17 bits of offset
    if (precision != GS_F64 && J > 14) return GS_ERR_UNSUPPORTED;
    for (int64_t i = 0; i < M * dim; ++i)
        if (!std::isfinite(xi[i])) return GS_ERR_BAD_NODES;
    if (mu)
        for (int64_t i = 0; i < M; ++i)
            if (!std::isfinite(mu[i]) || mu[i] < 0) return GS_ERR_BAD_NODES;

    std::unique_ptr<gs_plan_t> h;
    try {
        h.reset(new gs_plan_t());
    } catch (...) {
        return GS_ERR_NOMEM;
    }
    gs::Plan& P = h->impl;
    P.dim = dim; P.J = J; P.p = p; P.nb = (p == 1) ? 0 : p; P.N = 1 << J; P.M = M; P.precision = precision;
    // oversampling 2, except that the grid is never narrower than 16 cells:
    // every window (at most 14 taps) then covers distinct cells, so each grid
    // value enters a sum once (a wrapped window would sum it several times)
    P.ng = std::max(2 * P.N, gs::MIN_GRID);
    // Uniform nodes (Sec. 3.2): frequencies on a grid eps Z, eps = 2^-a, are
    // nodes of a grid of side N 2^a; on such nodes the transform is exact
    // (a zero-padded FFT read at the nodes, no window error)
    {
        const int a = uniform_level(xi, M * dim);
        const int64_t ng_max = dim == 2 ? 4096 : (int64_t)1 << 21;
        if (a >= 0 && std::max<int64_t>(P.ng, (int64_t)P.N << a) <= ng_max) {
            P.exact = true;
            P.ng = std::max(P.ng, P.N << a);
        }
    }
    P.G = gs::ilog2(P.ng);
    if (dim == 1 && P.ng > gs::FFT_MAX_LDS) {
        P.lg1 = P.G / 2; P.lg2 = P.G - P.lg1;
    } else {
        P.lg1 = P.G; P.lg2 = 0;
    }
    P.n1 = 1 << P.lg1; P.n2 = 1 << P.lg2;
    P.ts = std::min(gs::TILE, P.ng);
    if (dim == 2 && P.ts == gs::TILE) {
        P.cr1 = gs::colfft_r1(P.ng);
        P.cr2 = P.cr1 ? P.ng / P.cr1 : 0;
    }
    hipStream_t s = (hipStream_t)stream;

    try {
        (void)gs::basis_data(p);   // filters of this p (host construction, cached)
    } catch (const std::bad_alloc&) {
        return GS_ERR_NOMEM;
    } catch (...) {
        return GS_ERR_UNSUPPORTED;
    }

    // ---- device: point tables on the device, then the window, twiddle and workspace tables
    P.d64.present = precision == GS_F64 || precision == GS_F32_MIXED;
    P.d32.present = precision == GS_F32 || precision == GS_F32_MIXED;
    hipError_t e = hipSuccess;
    do {
        if ((e = gs::solver_alloc(P)) != hipSuccess) break;
        if ((e = gs::device_point_tables(P, xi, mu, s)) != hipSuccess) break;
        if (P.d64.present)
            if ((e = upload_prec<double>(P, gs::W64, gs::DEG64, 2.35 * gs::W64)) != hipSuccess) break;
        if (P.d32.present)
            if ((e = upload_prec<float>(P, gs::W32, gs::DEG32, 2.35 * gs::W32)) != hipSuccess) break;
        if (dim == 2 && P.nb > 0) {
            if ((e = hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking)) != hipSuccess) break;
            if ((e = hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming)) != hipSuccess) break;
            if ((e = hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming)) != hipSuccess) break;
        }
    } while (0);
    if (e != hipSuccess) {
        free_plan(P);
        return e == hipErrorOutOfMemory ? GS_ERR_NOMEM : hip_fail(e);
    }
    *out = h.release();
    return GS_OK;
}

int gs_plan_batch(gs_plan_t** out, int count, const gs_plan_desc* descs, void* stream) {
    if (!out || !descs || count < 1) return GS_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) out[i] = nullptr;
    for (int i = 0; i < count; ++i) {
        const gs_plan_desc& d = descs[i];
        const int rc = gs_plan(&out[i], d.dim, d.J, d.p, d.M, d.xi, d.mu, d.precision, stream);
        if (rc != GS_OK) {
            for (int k = 0; k < i; ++k) {
                gs_destroy(out[k]);
                out[k] = nullptr;
            }
            out[i] = nullptr;
            return rc;
        }
    }
    return GS_OK;
}

void gs_destroy(gs_plan_t* plan) {
    if (!plan) return;
    free_plan(plan->impl);
    delete plan;
}

static int pick_apply(const gs_plan_t* plan, const void* a, const void* b, int flags, bool& use64) {
    if (!plan || !a || !b) return GS_ERR_INVALID_ARG;
    if (flags & ~(GS_WEIGHTED | GS_SORTED | GS_APPLY_F64 | GS_WEIGHT_FULL)) return GS_ERR_INVALID_ARG;
    if ((flags & GS_WEIGHT_FULL) && !(flags & GS_WEIGHTED)) return GS_ERR_INVALID_ARG;
    const gs::Plan& P = plan->impl;
    if (P.precision == GS_F64) use64 = true;
    else if (P.precision == GS_F32) {
        if (flags & GS_APPLY_F64) return GS_ERR_PRECISION;
        use64 = false;
    } else use64 = (flags & GS_APPLY_F64) != 0;
    return GS_OK;
}

int gs_apply_T(const gs_plan_t* plan, const void* x, void* y, int flags, void* stream) {
    bool use64 = false;
    int rc = pick_apply(plan, x, y, flags, use64);
    if (rc) return rc;
    hipError_t e = use64 ? gs::launch_apply_T<double>(plan->impl, (const gs::cx<double>*)x, (gs::cx<double>*)y, flags,
                                                      (hipStream_t)stream)
                         : gs::launch_apply_T<float>(plan->impl, (const gs::cx<float>*)x, (gs::cx<float>*)y, flags,
                                                     (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e);
}

int gs_apply_TH(const gs_plan_t* plan, const void* u, void* x, int flags, void* stream) {
    bool use64 = false;
    int rc = pick_apply(plan, u, x, flags, use64);
    if (rc) return rc;
    hipError_t e = use64 ? gs::launch_apply_TH<double>(plan->impl, (const gs::cx<double>*)u, (gs::cx<double>*)x,
                                                       flags, (hipStream_t)stream)
                         : gs::launch_apply_TH<float>(plan->impl, (const gs::cx<float>*)u, (gs::cx<float>*)x, flags,
                                                      (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free adjoint
//
// gs_apply_TH_noalloc runs the adjoint's kernels on a workspace carved from
// one file-scope device array instead of the plan's own buffers.  Each device
// holds its own copy of the array; its device address is looked up once per
// device (with that device current) and cached.  Nothing in the array needs
// to start at zero: every kernel writes each workspace element before any
// kernel reads it (tile partials are written whole, empty tiles as zeros).
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};   // per device: device address of `scratch`

int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return GS_OK;
}

// Lays the adjoint workspace of plan P (precision T) out from `base` in
// 256-byte aligned pieces; returns the bytes it spans.  With base == 0 only
// the size is computed.
template <class T>
size_t carve_work(const gs::Plan& P, uintptr_t base, gs::Work<T>* w) {
    using C = gs::cx<T>;
    size_t off = 0;
    auto take = [&](size_t elems) -> C* {
        C* ptr = base ? reinterpret_cast<C*>(base + off) : nullptr;
        off += (elems * sizeof(C) + 255) & ~size_t(255);
        return ptr;
    };
    const size_t gsz = P.dim == 2 ? (size_t)P.ng * P.ng : (size_t)P.ng;
    gs::Work<T> r;
    r.grid = take(gsz);
    if (P.dim == 2 && P.nb) {
        r.sr = take((size_t)2 * P.nb * P.ng);
        r.sc = take((size_t)2 * P.nb * P.ng);
    }
    r.part = take(gs::adjoint_part_elems(P.dim, P.M, P.nb, P.ng));
    r.vbuf = take((size_t)P.M);
    if (w) *w = r;
    return off;
}

template <class T>
int apply_TH_static(const gs::Plan& P, const void* u, void* x, int flags, hipStream_t s) {
    const size_t need = carve_work<T>(P, 0, nullptr);
    if (need > (size_t)GS_NOALLOC_SCRATCH_BYTES) return GS_ERR_TOO_LARGE;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    gs::Work<T> w;
    carve_work<T>(P, reinterpret_cast<uintptr_t>(base), &w);
    hipError_t e = gs::launch_apply_TH<T>(P, (const gs::cx<T>*)u, (gs::cx<T>*)x, flags, s, &w);
    return e == hipSuccess ? GS_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int gs_apply_TH_noalloc(const gs_plan_t* plan, const void* u, void* x, int flags, void* stream) {
    bool use64 = false;
    int rc = pick_apply(plan, u, x, flags, use64);
    if (rc) return rc;
    return use64 ? apply_TH_static<double>(plan->impl, u, x, flags, (hipStream_t)stream)
                 : apply_TH_static<float>(plan->impl, u, x, flags, (hipStream_t)stream);
}

int gs_get_plan_info(const gs_plan_t* plan, gs_plan_info* info) {
    if (!plan || !info) return GS_ERR_INVALID_ARG;
    const gs::Plan& P = plan->impl;
    info->dim = P.dim; info->J = P.J; info->p = P.p; info->N = P.N; info->precision = P.precision;
    info->M = P.M; info->grid_n = P.ng;
    info->window_w32 = P.d32.present ? P.d32.w : 0;
    info->window_w64 = P.d64.present ? P.d64.w : 0;
    info->device_bytes = P.bytes;
    info->exact_nodes = P.exact ? 1 : 0;
    return GS_OK;
}

int gs_get_channels(const gs_plan_t* plan, int dimension, int f64, void* host_out) {
    if (!plan || !host_out) return GS_ERR_INVALID_ARG;
    const gs::Plan& P = plan->impl;
    if (dimension < 0 || dimension >= P.dim) return GS_ERR_INVALID_ARG;
    const size_t n = (size_t)(2 * P.nb + 1) * P.M;
    hipError_t e;
    if (f64) {
        if (!P.d64.present) return GS_ERR_PRECISION;
        e = hipMemcpy(host_out, dimension == 0 ? P.d64.chx : P.d64.chy, n * sizeof(gs::cx<double>),
                      hipMemcpyDeviceToHost);
    } else {
        if (!P.d32.present) return GS_ERR_PRECISION;
        e = hipMemcpy(host_out, dimension == 0 ? P.d32.chx : P.d32.chy, n * sizeof(gs::cx<float>),
                      hipMemcpyDeviceToHost);
    }
    return e == hipSuccess ? GS_OK : hip_fail(e);
}

int gs_get_permutation(const gs_plan_t* plan, int32_t* perm_host) {
    if (!plan || !perm_host) return GS_ERR_INVALID_ARG;
    hipError_t e = hipMemcpy(perm_host, plan->impl.perm, plan->impl.M * sizeof(int32_t), hipMemcpyDeviceToHost);
    return e == hipSuccess ? GS_OK : hip_fail(e);
}

int gs_profile_enable(int enable) {
    std::lock_guard<std::mutex> lk(gs::g_prof_mu);
    gs::prof_clear();
    gs::g_prof_enabled = enable != 0;
    return GS_OK;
}

int gs_profile_read(int max_kernels, char* names, int64_t* counts, double* total_ms, int* n_kernels) {
    if (!names || !counts || !total_ms || !n_kernels || max_kernels < 1) return GS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(gs::g_prof_mu);
    int64_t cnt[gs::K_COUNT] = {0};
    double tot[gs::K_COUNT] = {0};
    for (auto& r : gs::g_prof_recs) {
        if (!r.a || !r.b) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e);
        float ms = 0;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e);
        cnt[r.id] += 1;
        tot[r.id] += ms;
    }
    int n = 0;
    for (int k = 0; k < gs::K_COUNT && n < max_kernels; ++k) {
        if (!cnt[k]) continue;
        std::snprintf(names + 32 * n, 32, "%s", gs::kKernelNames[k]);
        counts[n] = cnt[k];
        total_ms[n] = tot[k];
        ++n;
    }
    *n_kernels = n;
    return GS_OK;
}

int gs_filter_taps(int p, double* h) {
    if (!h) return GS_ERR_INVALID_ARG;
    try {
        const gs::BasisData& b = gs::basis_data(p);
        std::copy(b.taps.begin(), b.taps.end(), h);
    } catch (...) {
        return GS_ERR_UNSUPPORTED;
    }
    return GS_OK;
}

int gs_boundary_filters(int p, double* U_left, double* V_left, double* v0_left, double* U_right, double* V_right,
                        double* v0_right) {
    if (p < 2) return GS_ERR_UNSUPPORTED;
    try {
        const gs::BasisData& b = gs::basis_data(p);
        if (U_left) std::copy(b.left.U.begin(), b.left.U.end(), U_left);
        if (V_left) std::copy(b.left.V.begin(), b.left.V.end(), V_left);
        if (v0_left) std::copy(b.left.v0.begin(), b.left.v0.end(), v0_left);
        if (U_right) std::copy(b.right.U.begin(), b.right.U.end(), U_right);
        if (V_right) std::copy(b.right.V.begin(), b.right.V.end(), V_right);
        if (v0_right) std::copy(b.right.v0.begin(), b.right.v0.end(), v0_right);
    } catch (...) {
        return GS_ERR_UNSUPPORTED;
    }
    return GS_OK;
}

int gs_eval_basis_1d(int J, int p, int64_t M, const double* xi, double* out) {
    if (!xi || !out || M < 0) return GS_ERR_INVALID_ARG;
    if (p < 1 || p > 8 || J < 1 || J > 30 || (1LL << J) < 2 * p) return GS_ERR_UNSUPPORTED;
    for (int64_t i = 0; i < M; ++i)
        if (!std::isfinite(xi[i])) return GS_ERR_BAD_NODES;
    try {
        gs::eval_basis_1d(J, p, M, xi, 1, reinterpret_cast<gs::cd*>(out), hw_threads());
    } catch (...) {
        return GS_ERR_UNSUPPORTED;
    }
    return GS_OK;
}

}  // extern "C"
