// Shared device/host definitions for libgs (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gs.h"

namespace gs {

// ------------------------------------------------------------ complex math
template <class T> struct alignas(2 * sizeof(T)) cx { T x, y; };
template <class T> using C_t = cx<T>;

// fixed-point position of the wrapped node eta' = frac(2^-J xi) in [0, 1)
template <class T> struct posw;
template <> struct posw<float> { using type = uint32_t; static constexpr int bits = 32; };
template <> struct posw<double> { using type = uint64_t; static constexpr int bits = 64; };
template <class T> using P_t = typename posw<T>::type;

template <class T> __host__ __device__ inline cx<T> mk(T a, T b) { cx<T> c; c.x = a; c.y = b; return c; }
template <class T> __host__ __device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <class T> __host__ __device__ inline cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <class T> __host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) { return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <class T> __host__ __device__ inline cx<T> conjc(cx<T> a) { return mk<T>(a.x, -a.y); }
template <class T> __host__ __device__ inline cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <class T> __host__ __device__ inline cx<T> cfma(cx<T> acc, cx<T> a, T s) { return mk<T>(acc.x + a.x * s, acc.y + a.y * s); }
template <class T> __host__ __device__ inline cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {  // acc + a*b
    return mk<T>(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
template <class T> __host__ __device__ inline cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b) {  // acc + conj(a)*b
    return mk<T>(acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x);
}
template <class T> __host__ __device__ inline cx<T> czero() { return mk<T>(T(0), T(0)); }

// per-point weight factor of a weighted apply: sqrt(mu), or mu with GS_WEIGHT_FULL
template <class T> __host__ __device__ inline T wscale(T smu, int flags) {
    return (flags & GS_WEIGHT_FULL) ? smu * smu : smu;
}

// ------------------------------------------------------------ plan
// Window / NFFT parameters per precision.
constexpr int W32 = 8, DEG32 = 7;     // FP32 path: 8 taps, degree-7 polynomial
constexpr int W64 = 14, DEG64 = 13;   // FP64 path: 14 taps, degree-13 polynomial

template <class T>
struct PrecData {
    using C = C_t<T>;
    using P = P_t<T>;
    bool present = false;
    int w = 0, deg = 0;
    P* pos = nullptr;      // [dim][M]
    C* chx = nullptr;      // [nch][M]
    C* chy = nullptr;      // [nch][M] (2D)
    T* smu = nullptr;      // [M]
    T* win = nullptr;      // [w][deg+1]
    T* deap = nullptr;     // [N]: 1 / KB-hat((n - N/2)/ng), zero at boundary columns
    C* tw = nullptr;       // [ng]: e^{-2 pi i k / ng}
    // workspace
    C* grid = nullptr;     // ng^dim (1D: four-step layout when ng > FFT_MAX_LDS)
    C* sr = nullptr;       // [2nb][ng]  2D row-side grids (along y)
    C* sc = nullptr;       // [2nb][ng]  2D col-side grids (along x)
    C* part = nullptr;     // partial sums
    C* vbuf = nullptr;     // [M] adjoint input in internal order (weighted)
    C* ybuf = nullptr;     // [M] apply output in internal order (solver)
    size_t part_elems = 0;
};

constexpr int FFT_MAX_LDS = 4096;   // largest single-pass FFT held in LDS
constexpr int MIN_GRID = 16;        // smallest NFFT grid side: at least the widest window
constexpr int TILE = 32;            // 2D point tiles: TILE x TILE grid cells

// sort key of a 2D cell: tile-major (tiles of ts x ts cells), row-major inside a tile
__host__ __device__ inline int64_t tile_key(int64_t cx, int64_t cy, int ts, int ng) {
    const int64_t ntx = ng / ts;
    return ((cx / ts) * ntx + (cy / ts)) * ts * ts + (cx % ts) * ts + (cy % ts);
}

struct Plan {
    int dim = 0, J = 0, p = 0, nb = 0, N = 0, precision = 0;
    int64_t M = 0;
    int ng = 0, G = 0;              // grid size per dim and log2
    bool exact = false;             // every node is a grid node: hat window, no deapodization
    int ts = 0;                     // 2D tile side in cells (min(TILE, ng))
    int n1 = 0, n2 = 0, lg1 = 0, lg2 = 0;   // four-step split (1D, ng > FFT_MAX_LDS)
    int cr1 = 0, cr2 = 0;           // 2D column transform split ng = cr1 * cr2 (0: natural row order);
                                    // frequency row k of the grid is stored in row cr2 * (k % cr1) + k / cr1
    int32_t* perm = nullptr;        // [M] internal -> caller index
    int32_t* cell_start = nullptr;  // [ng^dim + 1] points sorted by cell (row-major)
    int32_t* tile_order = nullptr;  // [tiles] 2D tiles in decreasing point count
    PrecData<double> d64;
    PrecData<float> d32;
    // solver state (device; FP64 vectors in internal point order)
    double* smu64 = nullptr;        // [M] sqrt(mu), internal order
    cx<double> *b = nullptr, *r = nullptr, *q = nullptr;     // [M]
    cx<double> *ps = nullptr, *ss = nullptr;                  // [N^dim]
    cx<float> *q32 = nullptr, *r32 = nullptr;                 // [M]   FP32-apply operands
    cx<float> *p32 = nullptr, *s32 = nullptr;                 // [N^dim]
    cx<double>* xbest = nullptr;    // [N^dim] best iterate of a reduced-precision recurrence
    double* red = nullptr;          // reduction partials [red_blocks]
    double* scal = nullptr;         // device scalars
    double* hist = nullptr;         // residual history (device)
    double* host_scal = nullptr;    // pinned host mirror of scal
    int red_blocks = 0, hist_len = 0;
    int64_t bytes = 0;
    std::string last_error;
    hipStream_t upload_stream = nullptr;
    // 2D adjoint: the column-side/corner kernel runs on `side` beside the
    // interior kernel (fork/join by events; serial while a graph is captured)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

template <class T> PrecData<T>& prec(Plan& p);
template <> inline PrecData<double>& prec<double>(Plan& p) { return p.d64; }
template <> inline PrecData<float>& prec<float>(Plan& p) { return p.d32; }
template <class T> const PrecData<T>& prec(const Plan& p);
template <> inline const PrecData<double>& prec<double>(const Plan& p) { return p.d64; }
template <> inline const PrecData<float>& prec<float>(const Plan& p) { return p.d32; }

// Transform workspace of one adjoint apply: the oversampled grid, the 2D side
// grids, the partial sums and the adjoint input in sorted order.  By default
// the plan's own buffers; the allocation-free entry point passes a carve-up of
// its static device array instead.
template <class T> struct Work {
    cx<T>* grid = nullptr;
    cx<T>* sr = nullptr;
    cx<T>* sc = nullptr;
    cx<T>* part = nullptr;
    cx<T>* vbuf = nullptr;
};
template <class T> inline Work<T> plan_work(const PrecData<T>& d) {
    Work<T> w;
    w.grid = d.grid; w.sr = d.sr; w.sc = d.sc; w.part = d.part; w.vbuf = d.vbuf;
    return w;
}

// ------------------------------------------------------------ launch modes
// Each launch site of the solver's iteration passes its kernel's per-problem
// arguments as one struct.  Normally (SINGLE) the kernel gets it by value.
// For batched solves the same launcher code first runs once per problem in
// RECORD mode (each site appends its struct; nothing is launched), then once
// per class of problems of equal geometry in BATCH mode: each site launches
// one kernel with gridDim.y = problem count, and the kernel reads problem
// blockIdx.y's struct from a device array.  Per problem, a batched kernel does
// exactly the arithmetic of the single launch.
struct LaunchCtx {
    enum Mode { SINGLE = 0, RECORD, BATCH };
    int mode = SINGLE;
    std::vector<std::vector<unsigned char>>* rec = nullptr;   // RECORD: per site, the structs
    const void* const* dev = nullptr;                         // BATCH: per site, device array
    const size_t* sizes = nullptr;                            // BATCH: per site, struct size
    int nsites = 0;
    int count = 0;                                            // BATCH: problems
    int site = 0;                                             // next site
};
extern thread_local LaunchCtx* g_launch;
inline bool launch_plain() { return !g_launch || g_launch->mode == LaunchCtx::SINGLE; }

// go(one, many, count) launches the kernel: many == nullptr for one problem
template <class A, class F>
inline hipError_t launch_site(const A& a, F&& go) {
    LaunchCtx* c = g_launch;
    if (!c || c->mode == LaunchCtx::SINGLE) return go(a, (const A*)nullptr, 1);
    const int i = c->site++;
    if (c->mode == LaunchCtx::RECORD) {
        if ((int)c->rec->size() <= i) c->rec->emplace_back();
        std::vector<unsigned char>& v = (*c->rec)[i];
        const unsigned char* b = reinterpret_cast<const unsigned char*>(&a);
        v.insert(v.end(), b, b + sizeof(A));
        return hipSuccess;
    }
    if (i >= c->nsites || c->sizes[i] != sizeof(A)) return hipErrorInvalidValue;
    return go(a, static_cast<const A*>(c->dev[i]), c->count);
}

// A kernel's per-problem arguments: `one` (by value) in the single-problem
// instance, else (BATCH) problem blockIdx.y's struct of the device array
// `many`, read word by word into scalar registers (every lane reads the same
// address).  The two instances share the kernel body, so a batched problem
// gets the single launch's arithmetic.
template <bool BATCH, class A>
__device__ __forceinline__ A kernel_args(const A& one, const A* __restrict__ many) {
    static_assert(sizeof(A) % 4 == 0, "argument structs are whole 32-bit words");
    if constexpr (!BATCH) {
        (void)many;
        return one;
    } else {
        uint32_t w[sizeof(A) / 4];
        const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(many + blockIdx.y);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(A) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
        A a;
        __builtin_memcpy(&a, w, sizeof(A));
        return a;
    }
}

template <class T> __device__ inline double sq64(cx<T> v) {
    const double a = (double)v.x, b = (double)v.y;
    return a * a + b * b;
}

// Deterministic workgroup sum (fixed shuffle tree per wavefront, then the
// wavefront sums in order); every thread gets the result
__device__ inline double wg_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    return s;
}

// launch helpers (defined in nfft.hip / fft.hip)
template <class T> hipError_t launch_apply_T(const Plan& P, const C_t<T>* x, C_t<T>* y, int flags, hipStream_t s);
// nsq: when non-null and norm_parts_TH(P) > 0, the adjoint also writes that
// many FP64 partial sums of |x_k|^2 (x as stored, in a fixed order) to nsq,
// so that ||x||^2 is their sum in index order.
template <class T> hipError_t launch_apply_TH(const Plan& P, const C_t<T>* u, C_t<T>* x, int flags, hipStream_t s,
                                              const Work<T>* work = nullptr, double* nsq = nullptr);
// number of partial sums launch_apply_TH writes to nsq (0: the path has none)
int norm_parts_TH(const Plan& P);

// column split of a 2D grid of side ng for the register column transform
// (0: single-pass LDS transform, natural row order)
inline int colfft_r1(int ng) { return ng == 1024 || ng == 512 ? 32 : (ng == 256 ? 16 : 0); }

inline int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

}  // namespace gs

struct gs_plan {
    gs::Plan impl;
};

#define GS_HIP_TRY(expr)                          \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return _e;          \
    } while (0)
static_assert(gs::MIN_GRID >= gs::W64 && gs::MIN_GRID >= gs::W32, "a window must fit the smallest grid");
