// 2D T and T^H with tile-staged kernels (Sec. 5, App. C; NFFT of Sec. 3.2).
//
// Points are sorted tile-major (tiles of TS x TS grid cells, row-major cells
// inside a tile), so the points of a tile are contiguous.
//
// Forward: interp_bnd_kernel evaluates the boundary part of each point (the
// four side blocks by 1D interpolation of the side grids, the four corner
// blocks densely) into a sorted-order buffer; interp_tile_kernel stages the
// tile's grid window (TS+W-1 squared) in LDS, interpolates the interior,
// adds the boundary part and applies D_x D_y and sqrt(mu).
//
// Adjoint: input in caller order is first gathered into sorted order and
// weighted (adj_gather_kernel; sorted input is weighted on the way in).  Two
// tile kernels then read the tile's points in chunks staged in LDS (window
// taps and channel products computed once per point):
//   * adj_interior_kernel: column-owner threads (one per padded output column
//     and block of cell rows) gather the interior 2D spread into register
//     accumulators, plus the row-side (x-boundary) channels;
//   * adj_boundary_kernel: four wavefronts sum the column-side (y-boundary)
//     channels per cell row and split the corner products
//     sum_m conj(ax_r ay_c) v_m among themselves as 16x16x4 MFMA steps.
// Each tile writes its partial padded grid, side and corner sums;
// merge_kernel adds the partials of neighbouring tiles in a fixed order (its
// first workgroups the grid blocks, the rest the side and corner entries).
// No atomics are used, and results are bitwise reproducible.
#include <algorithm>

#include "common.hpp"
#include "prof.hpp"

namespace gs {

template <class T>
struct TileGeo {
    int N, nb, ng, G, mask, M, ts, lts, ntx;
    int cr1, cr2;       // storage order of the transformed grid rows (see Plan::cr1)
    const P_t<T>* pos;
    const cx<T>* chx;
    const cx<T>* chy;
    const T* smu;
    const T* win;
    const int32_t* perm;
    const int32_t* cs;
    const int32_t* order;   // workgroup -> tile, heaviest tiles first
    __device__ int grow(int k) const { return cr1 ? cr2 * (k & (cr1 - 1)) + k / cr1 : k; }
    __device__ int bcol(int r) const { return r < nb ? r : N - 1 - (r - nb); }
    __device__ int bchan(int r) const { return r < nb ? r : r + 1; }
};

__device__ inline void decode_pos2(uint32_t u, int G, int& cell, float& t) {
    const int sh = 32 - G;
    cell = (int)(u >> sh);
    t = (float)(u & ((1u << sh) - 1u)) * __int_as_float((127 - sh) << 23);
}
__device__ inline void decode_pos2(uint64_t u, int G, int& cell, double& t) {
    const int sh = 64 - G;
    cell = (int)(u >> sh);
    t = (double)(u & ((1ull << sh) - 1ull)) * __longlong_as_double((long long)(1023 - sh) << 52);
}

// W window taps at fractional offset t in [0, 1): tap j = phi(t + W/2 - 1 - j),
// a degree-DEG polynomial p_j(x) in x = 2t - 1.  The window is even, so
// p_{W-1-j}(x) = p_j(-x): only the first W/2 polynomials are read, each split
// into even and odd parts in x^2, which gives both mirrored taps.
template <class T, int W, int DEG>
__device__ inline void taps_all(T t, const T* __restrict__ coef, T* w) {
    static_assert(W % 2 == 0, "even window width");
    constexpr int HE = DEG - (DEG & 1), HO = (DEG & 1) ? DEG : DEG - 1;
    const T x = T(2) * t - T(1), y = x * x;
#pragma unroll
    for (int j = 0; j < W / 2; ++j) {
        const T* c = coef + j * (DEG + 1);
        T e = c[HE];
#pragma unroll
        for (int i = HE - 2; i >= 0; i -= 2) e = e * y + c[i];
        T o = c[HO];
#pragma unroll
        for (int i = HO - 2; i >= 1; i -= 2) o = o * y + c[i];
        w[j] = e + x * o;
        w[W - 1 - j] = e - x * o;
    }
}

constexpr int TILE_TS = 32;     // grid cells per tile side
static_assert(TILE_TS == TILE, "tile side of the plan's sort");
constexpr int TILE_RB = 8;      // cell rows per column-owner block
// threads of the forward tile kernels, which loop over the tile's points: one
// point per thread on average in FP32, so that grids of few tiles (one
// workgroup per CU) still keep 16 waves per CU; FP64 keeps 256, its
// registers (up to 126) would not fit 1024-thread workgroups
template <class T> struct FwdThreads { static constexpr int value = 256; };
template <> struct FwdThreads<float> { static constexpr int value = 1024; };

// ------------------------------------------------------------------ forward

// Interior interpolation of one tile's points (plus the boundary part, when
// present, computed beforehand in sorted order), scales, weights and the
// scatter to caller order.
template <class T>
struct InterpTileArgs {
    TileGeo<T> g;
    const cx<T>* grid;
    const cx<T>* ybnd;
    cx<T>* y;
};

template <class T, int W, int DEG, bool BND>
__device__ __forceinline__ void interp_tile_kernel_body(const TileGeo<T>& g, const cx<T>* __restrict__ grid,
                                                        const cx<T>* __restrict__ ybnd, cx<T>* __restrict__ y,
                                                        int flags) {
    constexpr int TS = TILE_TS, PW = TS + W - 1;
    __shared__ cx<T> sG[PW * PW];
    const int tile = g.order[blockIdx.x];
    const int q0 = g.cs[tile << (2 * g.lts)];
    const int q1 = g.cs[(tile + 1) << (2 * g.lts)];
    if (q0 == q1) return;
    const int t0x = (tile / g.ntx) << g.lts, t0y = (tile % g.ntx) << g.lts;
    const int ox = t0x - (W / 2 - 1), oy = t0y - (W / 2 - 1);
    for (int e = threadIdx.x; e < PW * PW; e += blockDim.x) {
        const int i = e / PW, j = e - i * PW;
        sG[e] = grid[(size_t)g.grow((ox + i) & g.mask) * g.ng + ((oy + j) & g.mask)];
    }
    __syncthreads();
    const size_t M = g.M;
    const int nb = g.nb;
    for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        int cxg, cyg;
        T tx, ty;
        decode_pos2(g.pos[q], g.G, cxg, tx);
        decode_pos2(g.pos[M + q], g.G, cyg, ty);
        const int lx = cxg - t0x, ly = cyg - t0y;
        T wx[W], wy[W];
        taps_all<T, W, DEG>(tx, g.win, wx);
        taps_all<T, W, DEG>(ty, g.win, wy);
        cx<T> I = czero<T>();
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const cx<T>* row = sG + (lx + a) * PW + ly;
            cx<T> acc = czero<T>();
#pragma unroll
            for (int b = 0; b < W; ++b) acc = cfma(acc, row[b], wy[b]);
            I = cfma(I, acc, wx[a]);
        }
        cx<T> res = cmul(cmul(g.chx[nb * M + q], g.chy[nb * M + q]), I);
        if constexpr (BND) res = cadd(res, ybnd[q]);
        if (flags & GS_WEIGHTED) res = cscale(res, wscale(g.smu[q], flags));
        y[(flags & GS_SORTED) ? q : g.perm[q]] = res;
    }
}

template <class T, int W, int DEG, bool BND, bool BATCH>
__global__ void __launch_bounds__(FwdThreads<T>::value) interp_tile_kernel(InterpTileArgs<T> one,
                                                                           const InterpTileArgs<T>* many, int flags) {
    if constexpr (BATCH) {
        const InterpTileArgs<T> a = kernel_args<true>(one, many);
        interp_tile_kernel_body<T, W, DEG, BND>(a.g, a.grid, a.ybnd, a.y, flags);
    } else {
        interp_tile_kernel_body<T, W, DEG, BND>(one.g, one.grid, one.ybnd, one.y, flags);
    }
}

// Boundary part of T x for one tile's points (App. C): with ax_r, ay_c the
// boundary channels of the point and Dx, Dy its interior scales,
//   ybnd = Dy sum_r ax_r S_r + Dx sum_c ay_c C_c + sum_r ax_r sum_c X[r][c] ay_c,
// S_r the 1D interpolation (along y) of the row-side grid r and C_c that of the
// column-side grid c (along x).  Written in sorted order; the interior kernel adds it.
template <class T>
struct InterpBndArgs {
    TileGeo<T> g;
    const cx<T>* sr;
    const cx<T>* sc;
    const cx<T>* X;
    cx<T>* ybnd;
};

template <class T, int W, int DEG, int NB>
__device__ __forceinline__ void interp_bnd_kernel_body(const TileGeo<T>& g, const cx<T>* __restrict__ sr,
                                                       const cx<T>* __restrict__ sc, const cx<T>* __restrict__ X,
                                                       cx<T>* __restrict__ ybnd) {
    constexpr int TS = TILE_TS, PW = TS + W - 1, NCH = 2 * NB;
    __shared__ cx<T> sSR[NCH * PW];
    __shared__ cx<T> sSC[NCH * PW];
    __shared__ cx<T> sXC[NCH * NCH];
    const int tile = g.order[blockIdx.x];
    const int q0 = g.cs[tile << (2 * g.lts)];
    const int q1 = g.cs[(tile + 1) << (2 * g.lts)];
    if (q0 == q1) return;
    const int t0x = (tile / g.ntx) << g.lts, t0y = (tile % g.ntx) << g.lts;
    const int ox = t0x - (W / 2 - 1), oy = t0y - (W / 2 - 1);
    for (int e = threadIdx.x; e < NCH * PW; e += blockDim.x) {
        const int r = e / PW, j = e - r * PW;
        sSR[e] = sr[(size_t)r * g.ng + ((oy + j) & g.mask)];
        sSC[e] = sc[(size_t)r * g.ng + ((ox + j) & g.mask)];
    }
    for (int e = threadIdx.x; e < NCH * NCH; e += blockDim.x) {
        const int r = e / NCH, c = e - r * NCH;
        sXC[e] = X[(size_t)g.bcol(r) * g.N + g.bcol(c)];
    }
    __syncthreads();
    const size_t M = g.M;
    for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        int cxg, cyg;
        T tx, ty;
        decode_pos2(g.pos[q], g.G, cxg, tx);
        decode_pos2(g.pos[M + q], g.G, cyg, ty);
        const int lx = cxg - t0x, ly = cyg - t0y;
        T w[W];
        // row sides: sum_r ax_r S_r
        taps_all<T, W, DEG>(ty, g.win, w);
        cx<T> sR = czero<T>();
#pragma unroll 2
        for (int r = 0; r < NCH; ++r) {
            const cx<T>* s = sSR + r * PW + ly;
            cx<T> S = czero<T>();
#pragma unroll
            for (int b = 0; b < W; ++b) S = cfma(S, s[b], w[b]);
            sR = cmac(sR, g.chx[(size_t)(r < NB ? r : r + 1) * M + q], S);
        }
        cx<T> res = cmul(g.chy[NB * M + q], sR);
        // column sides: sum_c ay_c C_c
        taps_all<T, W, DEG>(tx, g.win, w);
        cx<T> sC = czero<T>();
#pragma unroll 2
        for (int c = 0; c < NCH; ++c) {
            const cx<T>* s = sSC + c * PW + lx;
            cx<T> C = czero<T>();
#pragma unroll
            for (int a = 0; a < W; ++a) C = cfma(C, s[a], w[a]);
            sC = cmac(sC, g.chy[(size_t)(c < NB ? c : c + 1) * M + q], C);
        }
        res = cmac(res, g.chx[NB * M + q], sC);
        // corners: sum_r ax_r sum_c X[r][c] ay_c
        cx<T> ay[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) ay[c] = g.chy[(size_t)(c < NB ? c : c + 1) * M + q];
#pragma unroll 2
        for (int r = 0; r < NCH; ++r) {
            cx<T> t = czero<T>();
#pragma unroll
            for (int c = 0; c < NCH; ++c) t = cmac(t, sXC[r * NCH + c], ay[c]);
            res = cmac(res, g.chx[(size_t)(r < NB ? r : r + 1) * M + q], t);
        }
        ybnd[q] = res;
    }
}

template <class T, int W, int DEG, int NB, bool BATCH>
__global__ void __launch_bounds__(FwdThreads<T>::value) interp_bnd_kernel(InterpBndArgs<T> one,
                                                                          const InterpBndArgs<T>* many) {
    if constexpr (BATCH) {
        const InterpBndArgs<T> a = kernel_args<true>(one, many);
        interp_bnd_kernel_body<T, W, DEG, NB>(a.g, a.sr, a.sc, a.X, a.ybnd);
    } else {
        interp_bnd_kernel_body<T, W, DEG, NB>(one.g, one.sr, one.sc, one.X, one.ybnd);
    }
}

// ------------------------------------------------------------------ adjoint

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
template <class T> struct Mfma;
// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16]; it receives
// four entries of column l%16 of D, at rows 4*(l/16)+v (f32) or (l/16)+4*v (f64).
template <> struct Mfma<float> {
    using acc = v4f;
    __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    using acc = v4d;
    __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// Row blocks and chunks.  A tile's points are split into NRB = TS/ADJ_RB row
// blocks (ADJ_RB cell rows each, contiguous in the tile's order).  Chunk k
// stages, for every row block b, its points k*CHB .. k*CHB+CHB-1 into LDS slots
// b*CHB + i, so every row block (and every thread that owns outputs of it) gets
// work in every chunk whatever the distribution of points over the rows.
constexpr int ADJ_RB = 4;

struct RbRange {
    int lo, hi;   // tile-relative point range of row block b staged in this chunk
};
template <int CHB>
__device__ inline RbRange rb_range(const int* off, int b, int k) {
    constexpr int TS = TILE_TS, RB = ADJ_RB;
    const int lo = off[b * RB * TS] + k * CHB;
    return RbRange{lo, min(lo + CHB, off[(b + 1) * RB * TS])};
}
template <int CHB>
__device__ inline int rb_chunks(const int* off) {
    constexpr int TS = TILE_TS, RB = ADJ_RB, NRB = TS / RB;
    int n = 0;
    for (int b = 0; b < NRB; ++b) n = max(n, (off[(b + 1) * RB * TS] - off[b * RB * TS] + CHB - 1) / CHB);
    return n;
}
template <int CHB>
__device__ inline int rb_point(const int* off, int k, int s) {   // tile-relative point of slot s, or -1
    constexpr int TS = TILE_TS, RB = ADJ_RB;
    const int b = s / CHB, i = s - b * CHB;
    const int p = off[b * RB * TS] + k * CHB + i;
    return p < off[(b + 1) * RB * TS] ? p : -1;
}

// Adjoint input of sorted point q, read by the tile kernels: u in sorted
// order, times the weight factor of a weighted apply.  Input in caller order
// is first gathered into sorted order by adj_gather_kernel (a random gather
// inside the tile kernels' chunk loads measured slower than the extra pass).
template <class T>
__device__ inline cx<T> adj_input(const TileGeo<T>& g, const cx<T>* __restrict__ u, int flags, int q) {
    cx<T> v = u[q];
    if (flags & GS_WEIGHTED) v = cscale(v, wscale(g.smu[q], flags));
    return v;
}

template <class T>
struct GatherArgs {
    TileGeo<T> g;
    const cx<T>* u;
    cx<T>* vs;
};

template <class T>
__device__ __forceinline__ void adj_gather_kernel_body(const GatherArgs<T>& A, int flags) {
    const TileGeo<T>& g = A.g;
    const cx<T>* __restrict__ u = A.u;
    cx<T>* __restrict__ vs = A.vs;
    // four points per thread: their random reads of u are in flight together
    const int q0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (q0 >= g.M) return;
    const int n = min(4, g.M - q0);
    int m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = i < n ? g.perm[q0 + i] : 0;
    cx<T> v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = u[m[i]];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= n) break;
        cx<T> w = v[i];
        if (flags & GS_WEIGHTED) w = cscale(w, wscale(g.smu[q0 + i], flags));
        vs[q0 + i] = w;
    }
}

template <class T, bool BATCH>
__global__ void adj_gather_kernel(GatherArgs<T> one, const GatherArgs<T>* __restrict__ many, int flags) {
    if constexpr (BATCH) {
        const GatherArgs<T> a = kernel_args<true>(one, many);
        adj_gather_kernel_body<T>(a, flags);
    } else {
        adj_gather_kernel_body<T>(one, flags);
    }
}

// Staged bytes per workgroup.  Workgroups of more than four wavefronts run two
// per CU only while each holds at most about 52 KB of LDS (measured on MI355X:
// 51 KB runs two per CU, 59 KB one), so the interior kernel's staging area
// stays below that.
// The FP64 kernels run one workgroup per CU (registers), so they stage more.
#ifndef GS_ADJ_INT_STAGE
#define GS_ADJ_INT_STAGE (48 * 1024)
#endif
template <class T> constexpr int adj_int_stage() { return sizeof(T) == 8 ? 72 * 1024 : GS_ADJ_INT_STAGE; }

constexpr int adj_chb(int budget, int slot_bytes, int nrb, int lo, int hi, int mult) {
    int c = budget / (nrb * slot_bytes);
    c = c > hi ? hi : c;
    c -= c % mult;
    return c < lo ? lo : c;
}

// LDS row lengths padded to an odd number of 16-byte units, so that lanes
// reading consecutive points with 16-byte loads spread over all banks
constexpr int pad16odd(int bytes) {
    int u = (bytes + 15) / 16;
    return 16 * (u | 1);
}
constexpr int pow2ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <int W>
struct IntShape {
    static constexpr int THREADS = ((TILE_TS + W - 1) * (TILE_TS / ADJ_RB) + 63) / 64 * 64;
};

template <class T, int W, int NB>
struct AdjIntLDS {
    static constexpr int TS = TILE_TS, PW = TS + W - 1, NRB = TS / ADJ_RB, NCH = 2 * NB;
    // y taps stored rotated by the point's cell column: wyr[(b + cy) mod WR] = wy[b],
    // so the thread owning padded column ply reads wyr[ply mod WR] without knowing cy
    static constexpr int WR = pow2ceil(W);
    static constexpr int LX = pad16odd(W * sizeof(T)) / sizeof(T);
    static constexpr int LY = pad16odd(WR * sizeof(T)) / sizeof(T);
    static constexpr int LC = NCH > 0 ? pad16odd(NCH * sizeof(cx<T>)) / sizeof(cx<T>) : 1;
    static constexpr int SLOT = (int)(sizeof(cx<T>) + (LX + LY) * sizeof(T) + LC * sizeof(cx<T>));
    // at most one slot per thread: the next chunk's loads are held in registers
    static constexpr int CHB = adj_chb(adj_int_stage<T>(), SLOT, NRB, 8, IntShape<W>::THREADS / NRB, 2), CH = NRB * CHB;
    struct Stage {
        cx<T> v[CH];                  // conj(Dx Dy) sqrt(mu) u
        T wx[CH][LX];                 // point-major so a thread reads a point's taps with wide loads
        T wy[CH][LY];
        cx<T> cr[CH][LC];             // conj(ax_r Dy) sqrt(mu) u: row-side values
    };
    struct Out {
        cx<T> P[PW][PW];
        cx<T> PR[NCH > 0 ? NCH : 1][PW];
    };
    static constexpr size_t bytes = sizeof(Stage) > sizeof(Out) ? sizeof(Stage) : sizeof(Out);
};

// global data of one staged point, loaded a chunk ahead
template <class T, int NB>
struct IntPre {
    int p;                       // tile-relative point, or -1 for an empty slot
    P_t<T> px, py;
    cx<T> v, dx, dy;
    cx<T> ax[NB > 0 ? 2 * NB : 1];
};

// Interior spread and row sides of one tile.  Thread (ply, rb) owns padded
// column ply for the output rows of row block rb (RB+W-1 register
// accumulators) and the row-side sums PR[r][ply] of the block (the x-boundary
// channels, spread along y); it gathers every point of the block whose cell
// column lies in [ply-W+1, ply], reading each point once per column.  The
// global loads of chunk k+1 are issued before chunk k is gathered.
template <class T>
struct AdjArgs {
    TileGeo<T> g;
    const cx<T>* u;
    cx<T>* part0;   // interior: grid partials; boundary: column-side partials
    cx<T>* part1;   // interior: row-side partials; boundary: corner partials
};

template <class T, int W, int DEG, int NB>
__device__ __forceinline__ void adj_interior_kernel_body(const AdjArgs<T>& A, int flags) {
    const TileGeo<T>& g = A.g;
    const cx<T>* __restrict__ u = A.u;
    cx<T>* __restrict__ partI = A.part0;
    cx<T>* __restrict__ partR = A.part1;
    using L = AdjIntLDS<T, W, NB>;
    constexpr int TS = TILE_TS, RB = ADJ_RB, PW = L::PW, NRB = L::NRB, CH = L::CH, CHB = L::CHB, NCH = L::NCH;
    constexpr int NACC = RB + W - 1;
    constexpr int NROUND = (NACC + RB - 1) / RB;   // row blocks b, b+NROUND write disjoint rows
    constexpr int NTHR = IntShape<W>::THREADS;
    static_assert(CH <= NTHR, "one slot per thread");
    __shared__ int off[TS * TS + 1];
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[L::bytes];
    auto& S = *reinterpret_cast<typename L::Stage*>(lds_raw);

    const int tile = g.order[blockIdx.x], tid = threadIdx.x;
    const int kbase = tile << (2 * g.lts);
    const int q0 = g.cs[kbase];
    const int t0y = (tile % g.ntx) << g.lts;
    for (int c = tid; c <= TS * TS; c += NTHR) off[c] = g.cs[kbase + c] - q0;
    __syncthreads();
    const int nck = rb_chunks<CHB>(off);
    const size_t M = g.M;
    const int ply = tid % PW, rb = tid / PW;
    const bool act = rb < NRB;
    const int cy_lo = max(0, ply - (W - 1)), cy_hi = min(TS - 1, ply);

    IntPre<T, NB> pre;
    auto load = [&](int k) {
        pre.p = tid < CH ? rb_point<CHB>(off, k, tid) : -1;
        if (pre.p < 0) return;
        const int q = q0 + pre.p;
        pre.px = g.pos[q];
        pre.py = g.pos[M + q];
        pre.v = adj_input(g, u, flags, q);
        pre.dx = g.chx[NB * M + q];
        pre.dy = g.chy[NB * M + q];
#pragma unroll
        for (int r = 0; r < NCH; ++r) pre.ax[r] = g.chx[(size_t)(r < NB ? r : r + 1) * M + q];
    };
    if (nck > 0) load(0);

    cx<T> acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = czero<T>();
    cx<T> accR[NCH > 0 ? NCH : 1];
#pragma unroll
    for (int i = 0; i < (NCH > 0 ? NCH : 1); ++i) accR[i] = czero<T>();

    for (int k = 0; k < nck; ++k) {
        if (k) __syncthreads();
        if (pre.p >= 0) {
            const int s = tid;
            int cxg, cyg;
            T tx, ty;
            decode_pos2(pre.px, g.G, cxg, tx);
            decode_pos2(pre.py, g.G, cyg, ty);
            S.v[s] = cmul(conjc(cmul(pre.dx, pre.dy)), pre.v);
            const int rot = cyg - t0y;
            T w[W];
            taps_all<T, W, DEG>(tx, g.win, w);
#pragma unroll
            for (int j = 0; j < W; ++j) S.wx[s][j] = w[j];
            taps_all<T, W, DEG>(ty, g.win, w);
#pragma unroll
            for (int j = 0; j < W; ++j) S.wy[s][(j + rot) & (L::WR - 1)] = w[j];
            if constexpr (NB > 0) {
                const cx<T> vy = cmul(conjc(pre.dy), pre.v);
#pragma unroll
                for (int c = 0; c < NCH; ++c) S.cr[s][c] = cmul(conjc(pre.ax[c]), vy);
            }
        }
        __syncthreads();
        if (k + 1 < nck) load(k + 1);
        if (act) {
            const RbRange R = rb_range<CHB>(off, rb, k);
            const int sb = rb * CHB - R.lo;
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int row = rb * RB + rr;
                const int pa = max(off[row * TS + cy_lo], R.lo), pb = min(off[row * TS + cy_hi + 1], R.hi);
                for (int p = pa; p < pb; ++p) {
                    const int t = sb + p;
                    const T w = S.wy[t][ply & (L::WR - 1)];
                    const cx<T> tv = cscale(S.v[t], w);
                    T wx[W];
#pragma unroll
                    for (int a = 0; a < W; ++a) wx[a] = S.wx[t][a];
#pragma unroll
                    for (int a = 0; a < W; ++a) acc[rr + a] = cfma(acc[rr + a], tv, wx[a]);
                    if constexpr (NB > 0) {
                        cx<T> cr[NCH];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) cr[c] = S.cr[t][c];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) accR[c] = cfma(accR[c], cr[c], w);
                    }
                }
            }
        }
    }
    __syncthreads();
    auto& O = *reinterpret_cast<typename L::Out*>(lds_raw);
    for (int e = tid; e < PW * PW; e += NTHR) (&O.P[0][0])[e] = czero<T>();
    if constexpr (NB > 0)
        for (int e = tid; e < NCH * PW; e += NTHR) (&O.PR[0][0])[e] = czero<T>();
    __syncthreads();
    // row blocks overlap in W-1 output rows: add them in NROUND fixed rounds
    for (int r = 0; r < NROUND; ++r) {
        if (act && rb % NROUND == r) {
#pragma unroll
            for (int i = 0; i < NACC; ++i) O.P[rb * RB + i][ply] = cadd(O.P[rb * RB + i][ply], acc[i]);
        }
        __syncthreads();
    }
    if constexpr (NB > 0) {
        for (int r = 0; r < NRB; ++r) {
            if (act && rb == r) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) O.PR[c][ply] = cadd(O.PR[c][ply], accR[c]);
            }
            __syncthreads();
        }
        cx<T>* pR = partR + (size_t)tile * NCH * PW;
        for (int e = tid; e < NCH * PW; e += NTHR) pR[e] = (&O.PR[0][0])[e];
    }
    cx<T>* pI = partI + (size_t)tile * PW * PW;
    for (int e = tid; e < PW * PW; e += NTHR) pI[e] = (&O.P[0][0])[e];
}

template <class T, int W, int DEG, int NB, bool BATCH>
__global__ void __launch_bounds__(IntShape<W>::THREADS) adj_interior_kernel(AdjArgs<T> one, const AdjArgs<T>* __restrict__ many,
                                                                            int flags) {
    if constexpr (BATCH) {
        const AdjArgs<T> a = kernel_args<true>(one, many);
        adj_interior_kernel_body<T, W, DEG, NB>(a, flags);
    } else {
        adj_interior_kernel_body<T, W, DEG, NB>(one, flags);
    }
}

// Column sides and corners of one tile (App. C, the remaining blocks of the
// 2D matrix), with the same row-block chunked staging as the interior kernel.
// Four wavefronts; each one
//   * stages half-slots of the chunk (x taps and x channels, or the y channels),
//   * walks two row blocks of the chunk for the column sides
//     PC[c][x] = sum_m dc_c(m) wx_m[x - cx_m]: with lane = (c, a) it sums, per
//     cell row, B[c][a] = sum over the row's points of dc_c wx[a] and adds B to
//     its own partial at (c, row + a); all lanes walk the same points, so the
//     work is balanced whatever the distribution of points,
//   * runs a quarter of the corner products sum_m conj(ax_r ay_c) sqrt(mu_m) u_m
//     as real 16x16x4 MFMA steps over the chunk's slots.
// Workgroups of four wavefronts run two per CU with up to 80 KB of LDS each,
// four per CU with up to 40 KB.  The stage budget is a template parameter:
// FP32 on grids of more than 256 tiles stages 12 points per row block (about
// 40 KB, four workgroups per CU: 73 against 78 us with the 76 KB stage at the
// 1,048,576-point J = 9 workload); on smaller grids, where the kernel runs
// beside the interior kernel, and in FP64 the stage fills 76 KB.
constexpr int BND_WAVES = 4;
constexpr int BND_THREADS = 64 * BND_WAVES;
constexpr int BND_LDS = 76 * 1024;
constexpr int BND_LDS_FOUR = 40 * 1024;

template <class T, int W, int NB, int BL = BND_LDS>
struct AdjBndLDS {
    static constexpr int TS = TILE_TS, PW = TS + W - 1, NRB = TS / ADJ_RB;
    static constexpr int NCH = 2 * NB, NE = 4 * NB;          // channels; real entries of e, f
    static constexpr int NBLK = (NE + 15) / 16;               // 16x16 MFMA blocks per side
    static constexpr int LD = 16 * NBLK;
    static constexpr int FIXED = (int)(4 * (TS * TS + 1) + BND_WAVES * NCH * PW * sizeof(cx<T>) +
                                       BND_WAVES * LD * LD * sizeof(T));
    static constexpr int SLOT = (int)(W * sizeof(T) + NCH * sizeof(cx<T>) + 2 * NE * sizeof(T));
    static constexpr int CHB = adj_chb(BL - FIXED, SLOT, NRB, 4, 32, 4), CH = NRB * CHB;
    struct Stage {
        T wx[CH][W];
        cx<T> dc[CH][NCH];   // conj(ay_c Dx) sqrt(mu) u: column-side values
        T e[CH][NE];         // re / im of conj(ax_r) sqrt(mu) u
        T f[CH][NE];         // re / -im of ay_c
    };
};

// global data of one staged point, loaded a chunk ahead, split over two
// threads: half 0 takes the x coordinate and x channels, half 1 the y channels
template <class T, int NB>
struct BndPre {
    int p;
    P_t<T> px;
    cx<T> v, d;
    cx<T> ch[2 * NB];
};

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class T, int W, int DEG, int NB, int BL>
__device__ __forceinline__ void adj_boundary_kernel_body(const AdjArgs<T>& A, int flags) {
    const TileGeo<T>& g = A.g;
    const cx<T>* __restrict__ u = A.u;
    cx<T>* __restrict__ partC = A.part0;
    cx<T>* __restrict__ partX = A.part1;
    using L = AdjBndLDS<T, W, NB, BL>;
    constexpr int TS = TILE_TS, RB = ADJ_RB, PW = L::PW, NRB = L::NRB, NCH = L::NCH, NE = L::NE;
    constexpr int CH = L::CH, CHB = L::CHB;
    constexpr int NBLK = L::NBLK, LD = L::LD;
    constexpr int NPAIR = NCH * W, NPB = (NPAIR + 63) / 64;   // (channel, tap) lanes and their wave blocks
    static_assert(NPB <= BND_WAVES, "column-side lanes");
    constexpr int RG = BND_WAVES / NPB;                       // row-block groups
    constexpr int NCHAIN = (NRB + RG - 1) / RG;               // row blocks per wavefront
    constexpr int HPT = (2 * CH + BND_THREADS - 1) / BND_THREADS;   // half-slots per thread
    __shared__ int off[TS * TS + 1];
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[sizeof(typename L::Stage)];
    __shared__ cx<T> PCw[BND_WAVES][NCH][PW];
    __shared__ T cbuf[BND_WAVES][LD * LD];
    __shared__ T swin[(W / 2) * (DEG + 1)];   // the W/2 tap polynomials the symmetric evaluation reads
    auto& S = *reinterpret_cast<typename L::Stage*>(lds_raw);

    const int tile = g.order[blockIdx.x], tid = threadIdx.x;
    const int kbase = tile << (2 * g.lts);
    const int q0 = g.cs[kbase];
    // array bases as locals: the half-slot selection below is then a register select
    const P_t<T>* __restrict__ gpos = g.pos;
    const cx<T>* __restrict__ gchx = g.chx;
    const cx<T>* __restrict__ gchy = g.chy;
    for (int c = tid; c <= TS * TS; c += BND_THREADS) off[c] = g.cs[kbase + c] - q0;
    for (int c = tid; c < (W / 2) * (DEG + 1); c += BND_THREADS) swin[c] = g.win[c];
    for (int e = tid; e < BND_WAVES * NCH * PW; e += BND_THREADS) (&PCw[0][0][0])[e] = czero<T>();
    __syncthreads();
    const int nck = rb_chunks<CHB>(off);
    const size_t M = g.M;
    const int wave = tid >> 6, lane = tid & 63;
    // column-side lane roles
    const int pb = wave % NPB, rg = wave / NPB;
    const int pair = pb * 64 + lane;
    const bool colact = rg < RG && pair < NPAIR;
    const int cc = pair / W, ca = pair - cc * W;
    cx<T> accC[NCHAIN];
    int cur[NCHAIN];     // cell row being summed per row block (uniform), -1 before the first
#pragma unroll
    for (int i = 0; i < NCHAIN; ++i) {
        accC[i] = czero<T>();
        cur[i] = -1;
    }
    // corner lane roles
    const int li = lane & 15, kk = lane >> 4;
    typename Mfma<T>::acc accM[NBLK * NBLK];
#pragma unroll
    for (int b = 0; b < NBLK * NBLK; ++b) accM[b] = Mfma<T>::zero();

    BndPre<T, NB> pre[HPT];
    auto load = [&](int k) {
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int h = tid + j * BND_THREADS;
            pre[j].p = h < 2 * CH ? rb_point<CHB>(off, k, h >> 1) : -1;
            if (pre[j].p < 0) continue;
            const int q = q0 + pre[j].p;
            const bool xh = (h & 1) == 0;
            pre[j].v = adj_input(g, u, flags, q);
            if (xh)
                pre[j].px = gpos[q];
            else
                pre[j].d = gchx[NB * M + q];
            const cx<T>* __restrict__ chp = xh ? gchx : gchy;
#pragma unroll
            for (int r = 0; r < NCH; ++r) pre[j].ch[r] = chp[(size_t)(r < NB ? r : r + 1) * M + q];
        }
    };
    if (nck > 0) load(0);

    for (int k = 0; k < nck; ++k) {
        if (k) __syncthreads();
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int h = tid + j * BND_THREADS;
            if (h >= 2 * CH) continue;
            const int s = h >> 1;
            const BndPre<T, NB>& P = pre[j];
            if (P.p < 0) {
                // empty slots enter the corner product as zeros
#pragma unroll
                for (int i = 0; i < NE; ++i) ((h & 1) == 0 ? S.e[s][i] : S.f[s][i]) = T(0);
            } else if ((h & 1) == 0) {
                int cxg;
                T tx;
                decode_pos2(P.px, g.G, cxg, tx);
                T w[W];
                taps_all<T, W, DEG>(tx, swin, w);
#pragma unroll
                for (int jj = 0; jj < W; ++jj) S.wx[s][jj] = w[jj];
#pragma unroll
                for (int r = 0; r < NCH; ++r) {
                    const cx<T> e = cmul(conjc(P.ch[r]), P.v);
                    S.e[s][r] = e.x;
                    S.e[s][NCH + r] = e.y;
                }
            } else {
                const cx<T> vx = cmul(conjc(P.d), P.v);
#pragma unroll
                for (int r = 0; r < NCH; ++r) {
                    S.dc[s][r] = cmul(conjc(P.ch[r]), vx);
                    S.f[s][r] = P.ch[r].x;
                    S.f[s][NCH + r] = -P.ch[r].y;
                }
            }
        }
        __syncthreads();
        if (k + 1 < nck) load(k + 1);
        if (colact) {
#pragma unroll
            for (int i = 0; i < NCHAIN; ++i) {
                const int b = rg + i * RG;
                if (b >= NRB) continue;
                const RbRange R = rb_range<CHB>(off, b, k);
                const int sb = b * CHB - R.lo;
                int p = uniform(R.lo);
                const int hi = uniform(R.hi);
                while (p < hi) {
                    // the cell row holding point p; rows are walked in increasing order
                    int row = cur[i] < 0 ? b * RB : cur[i];
                    while (uniform(off[(row + 1) * TS]) <= p) ++row;
                    if (row != cur[i]) {
                        if (cur[i] >= 0) PCw[wave][cc][cur[i] + ca] = cadd(PCw[wave][cc][cur[i] + ca], accC[i]);
                        accC[i] = czero<T>();
                        cur[i] = row;
                    }
                    const int pe = min(hi, uniform(off[(row + 1) * TS]));
                    // four interleaved partial sums, eight points per step: the loads of
                    // a step are issued together
                    cx<T> s0 = accC[i], s1 = czero<T>(), s2 = czero<T>(), s3 = czero<T>();
                    for (; p + 7 < pe; p += 8) {
                        cx<T> d[8];
                        T w[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            d[j] = S.dc[sb + p + j][cc];
                            w[j] = S.wx[sb + p + j][ca];
                        }
                        s0 = cfma(cfma(s0, d[0], w[0]), d[4], w[4]);
                        s1 = cfma(cfma(s1, d[1], w[1]), d[5], w[5]);
                        s2 = cfma(cfma(s2, d[2], w[2]), d[6], w[6]);
                        s3 = cfma(cfma(s3, d[3], w[3]), d[7], w[7]);
                    }
                    for (; p < pe; ++p) s0 = cfma(s0, S.dc[sb + p][cc], S.wx[sb + p][ca]);
                    accC[i] = cadd(cadd(s0, s1), cadd(s2, s3));
                }
            }
        }
        // this wavefront's share of the corner steps, 4 slots per MFMA step
        for (int s4 = wave; s4 < CH / 4; s4 += BND_WAVES) {
            const int t = 4 * s4 + kk;
#pragma unroll
            for (int bi = 0; bi < NBLK; ++bi) {
                const int ie = bi * 16 + li;
                const T av = ie < NE ? S.e[t][ie] : T(0);
#pragma unroll
                for (int bj = 0; bj < NBLK; ++bj) {
                    const int jf = bj * 16 + li;
                    const T bv = jf < NE ? S.f[t][jf] : T(0);
                    accM[bi * NBLK + bj] = Mfma<T>::step(av, bv, accM[bi * NBLK + bj]);
                }
            }
        }
    }
    if (colact) {
#pragma unroll
        for (int i = 0; i < NCHAIN; ++i)
            if (cur[i] >= 0) PCw[wave][cc][cur[i] + ca] = cadd(PCw[wave][cc][cur[i] + ca], accC[i]);
    }
#pragma unroll
    for (int bi = 0; bi < NBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBLK; ++bj)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const int row = bi * 16 + Mfma<T>::row(lane, vv), col = bj * 16 + (lane & 15);
                cbuf[wave][row * LD + col] = accM[bi * NBLK + bj][vv];
            }
    __syncthreads();
    // wavefront partials in fixed order
    cx<T>* pC = partC + (size_t)tile * NCH * PW;
    for (int e = tid; e < NCH * PW; e += BND_THREADS) {
        cx<T> s = (&PCw[0][0][0])[e];
#pragma unroll
        for (int w = 1; w < BND_WAVES; ++w) s = cadd(s, (&PCw[w][0][0])[e]);
        pC[e] = s;
    }
    cx<T>* pX = partX + (size_t)tile * NCH * NCH;
    for (int e = tid; e < NCH * NCH; e += BND_THREADS) {
        const int r = e / NCH, c = e - r * NCH;
        T re = T(0), im = T(0);
#pragma unroll
        for (int w = 0; w < BND_WAVES; ++w) {
            re += cbuf[w][r * LD + c] - cbuf[w][(NCH + r) * LD + NCH + c];
            im += cbuf[w][r * LD + NCH + c] + cbuf[w][(NCH + r) * LD + c];
        }
        pX[e] = mk<T>(re, im);
    }
}

template <class T, int W, int DEG, int NB, int BL, bool BATCH>
__global__ void __launch_bounds__(BND_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
adj_boundary_kernel(AdjArgs<T> one, const AdjArgs<T>* __restrict__ many, int flags) {
    if constexpr (BATCH) {
        const AdjArgs<T> a = kernel_args<true>(one, many);
        adj_boundary_kernel_body<T, W, DEG, NB, BL>(a, flags);
    } else {
        adj_boundary_kernel_body<T, W, DEG, NB, BL>(one, flags);
    }
}

// grid cell (gx, gy) = sum of the padded tile partials that cover it (fixed order)
template <class T>
struct MergeGridArgs {
    TileGeo<T> g;
    const cx<T>* partI;
    cx<T>* grid;
};

template <class T, int W>
__device__ __forceinline__ void merge_grid_kernel_body(const MergeGridArgs<T>& A, int bid) {
    const TileGeo<T>& g = A.g;
    const cx<T>* __restrict__ partI = A.partI;
    cx<T>* __restrict__ grid = A.grid;
    constexpr int TS = TILE_TS, PW = TS + W - 1, H = W / 2 - 1;
    const int idx = bid * blockDim.x + threadIdx.x;
    if (idx >= g.ng * g.ng) return;
    const int gx = idx >> g.G, gy = idx & g.mask;
    const int sx = (gx + H) & g.mask, sy = (gy + H) & g.mask;
    const int tx0 = sx >> g.lts, px0 = sx & (TS - 1);
    const int ty0 = sy >> g.lts, py0 = sy & (TS - 1);
    const bool ox = px0 < W - 1, oy = py0 < W - 1;
    const int txm = (tx0 + g.ntx - 1) % g.ntx, tym = (ty0 + g.ntx - 1) % g.ntx;
    cx<T> s = czero<T>();
    if (ox && oy) s = cadd(s, partI[(size_t)(txm * g.ntx + tym) * PW * PW + (px0 + TS) * PW + py0 + TS]);
    if (ox) s = cadd(s, partI[(size_t)(txm * g.ntx + ty0) * PW * PW + (px0 + TS) * PW + py0]);
    if (oy) s = cadd(s, partI[(size_t)(tx0 * g.ntx + tym) * PW * PW + px0 * PW + py0 + TS]);
    s = cadd(s, partI[(size_t)(tx0 * g.ntx + ty0) * PW * PW + px0 * PW + py0]);
    grid[idx] = s;
}

template <class T, int W, bool BATCH>
__global__ void merge_grid_kernel(MergeGridArgs<T> one, const MergeGridArgs<T>* __restrict__ many) {
    if constexpr (BATCH) {
        const MergeGridArgs<T> a = kernel_args<true>(one, many);
        merge_grid_kernel_body<T, W>(a, blockIdx.x);
    } else {
        merge_grid_kernel_body<T, W>(one, blockIdx.x);
    }
}

// Side grids and corners from the tile partials, in a fixed order.
//   blocks [0, nside): 32 positions gl of one side grid (row sides sr[r][gy]: the
//     tiles of tile column gy; column sides sc[c][gx]: the tiles of tile row gx),
//     8 thread groups each summing a fixed run of tiles, then the 8 group sums in order;
//   blocks [nside, nside + nch^2): one corner entry X[bcol(r)][bcol(c)] over all tiles.
constexpr int MERGE_GROUPS = 8;
template <class T>
struct MergeSidesArgs {
    TileGeo<T> g;
    const cx<T>* partR;
    const cx<T>* partC;
    const cx<T>* partX;
    cx<T>* sr;
    cx<T>* sc;
    cx<T>* X;
};

template <class T, int W>
__device__ __forceinline__ void merge_sides_kernel_body(const MergeSidesArgs<T>& A, int nside, int bid) {
    const TileGeo<T>& g = A.g;
    const cx<T>* __restrict__ partR = A.partR;
    const cx<T>* __restrict__ partC = A.partC;
    const cx<T>* __restrict__ partX = A.partX;
    cx<T>* __restrict__ sr = A.sr;
    cx<T>* __restrict__ sc = A.sc;
    cx<T>* __restrict__ X = A.X;
    constexpr int TS = TILE_TS, PW = TS + W - 1, H = W / 2 - 1;
    __shared__ cx<T> sh[256];
    const int nch = 2 * g.nb;
    const int tid = threadIdx.x;
    if (bid >= nside) {
        const int e = bid - nside;   // (r, c)
        const int nt = g.ntx * g.ntx;
        cx<T> s = czero<T>();
        for (int t = tid; t < nt; t += 256) s = cadd(s, partX[(size_t)t * nch * nch + e]);
        sh[tid] = s;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if (tid < k) sh[tid] = cadd(sh[tid], sh[tid + k]);
            __syncthreads();
        }
        if (tid == 0) X[(size_t)g.bcol(e / nch) * g.N + g.bcol(e % nch)] = sh[0];
        return;
    }
    const int per = g.ng / 32;                      // blocks per side grid
    const int which = bid / (nch * per);
    const int r = (bid / per) % nch;
    const int gl = (bid % per) * 32 + (tid & 31);
    const int grp = tid >> 5;
    const int sl = (gl + H) & g.mask;
    const int t0 = sl >> g.lts, p0 = sl & (TS - 1);
    const bool o = p0 < W - 1;
    const int tm = (t0 + g.ntx - 1) % g.ntx;
    const int tpg = (g.ntx + MERGE_GROUPS - 1) / MERGE_GROUPS;
    const int ta = grp * tpg, tb = min(g.ntx, ta + tpg);
    cx<T> s = czero<T>();
    if (which == 0) {   // row sides: tiles (t, t0) and (t, tm)
        for (int t = ta; t < tb; ++t) {
            if (o) s = cadd(s, partR[((size_t)(t * g.ntx + tm) * nch + r) * PW + p0 + TS]);
            s = cadd(s, partR[((size_t)(t * g.ntx + t0) * nch + r) * PW + p0]);
        }
    } else {            // column sides: tiles (t0, t) and (tm, t)
        for (int t = ta; t < tb; ++t) {
            if (o) s = cadd(s, partC[((size_t)(tm * g.ntx + t) * nch + r) * PW + p0 + TS]);
            s = cadd(s, partC[((size_t)(t0 * g.ntx + t) * nch + r) * PW + p0]);
        }
    }
    sh[tid] = s;
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int k = 1; k < MERGE_GROUPS; ++k) s = cadd(s, sh[k * 32 + tid]);
        (which == 0 ? sr : sc)[(size_t)r * g.ng + gl] = s;
    }
}

// Grid and side merges in one launch: blocks [0, ngrid) merge the grid, the
// rest the side grids and corners.
template <class T>
struct MergeArgs {
    MergeGridArgs<T> grid;
    MergeSidesArgs<T> sides;
};

template <class T, int W, bool BATCH>
__global__ void __launch_bounds__(256) merge_kernel(MergeArgs<T> one, const MergeArgs<T>* many, int ngrid,
                                                    int nside) {
    const int bid = blockIdx.x;
    if constexpr (BATCH) {
        const MergeArgs<T> a = kernel_args<true>(one, many);
        if (bid < ngrid) merge_grid_kernel_body<T, W>(a.grid, bid);
        else merge_sides_kernel_body<T, W>(a.sides, nside, bid - ngrid);
    } else {
        if (bid < ngrid) merge_grid_kernel_body<T, W>(one.grid, bid);
        else merge_sides_kernel_body<T, W>(one.sides, nside, bid - ngrid);
    }
}

// ------------------------------------------------------------------ launchers

template <class T>
TileGeo<T> make_tile_geo(const Plan& P) {
    const PrecData<T>& d = prec<T>(P);
    TileGeo<T> g;
    g.N = P.N; g.nb = P.nb; g.ng = P.ng; g.G = P.G; g.mask = P.ng - 1; g.M = (int)P.M;
    g.ts = P.ts; g.lts = ilog2(P.ts); g.ntx = P.ng / P.ts;
    g.cr1 = P.cr1; g.cr2 = P.cr2;
    g.pos = d.pos; g.chx = d.chx; g.chy = d.chy; g.smu = d.smu; g.win = d.win;
    g.perm = P.perm; g.cs = P.cell_start; g.order = P.tile_order;
    return g;
}

template <class T> struct TileWin;
template <> struct TileWin<float> { static constexpr int W = W32, DEG = DEG32; };
template <> struct TileWin<double> { static constexpr int W = W64, DEG = DEG64; };

template <class T, int NB>
hipError_t interp2d_tile_nb(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s, int part) {
    const PrecData<T>& d = prec<T>(P);
    const TileGeo<T> g = make_tile_geo<T>(P);
    constexpr int W = TileWin<T>::W, DEG = TileWin<T>::DEG;
    const int nt = g.ntx * g.ntx;
    if constexpr (NB > 0) if (part & 1) {
        ProfScope _p(K_INTERP_BND, s);
        using A = InterpBndArgs<T>;
        GS_HIP_TRY(launch_site(A{g, d.sr, d.sc, x, d.ybuf}, [&](const A& one, const A* many, int count) {
            if (many) hipLaunchKernelGGL((interp_bnd_kernel<T, W, DEG, NB, true>), dim3(nt, count), dim3(FwdThreads<T>::value), 0, s,
                               one, many);
        else hipLaunchKernelGGL((interp_bnd_kernel<T, W, DEG, NB, false>), dim3(nt, count), dim3(FwdThreads<T>::value), 0, s,
                               one, many);
            return hipGetLastError();
        }));
    }
    if (!(part & 2)) return hipSuccess;
    ProfScope _p(K_INTERP2D, s);
    using A = InterpTileArgs<T>;
    return launch_site(A{g, d.grid, d.ybuf, y}, [&](const A& one, const A* many, int count) {
        if (many) hipLaunchKernelGGL((interp_tile_kernel<T, W, DEG, (NB > 0), true>), dim3(nt, count), dim3(FwdThreads<T>::value), 0, s,
                           one, many, flags);
        else hipLaunchKernelGGL((interp_tile_kernel<T, W, DEG, (NB > 0), false>), dim3(nt, count), dim3(FwdThreads<T>::value), 0, s,
                           one, many, flags);
        return hipGetLastError();
    });
}

template <class T, int NB>
hipError_t adjoint2d_tile_nb(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s, const Work<T>& d) {
    const TileGeo<T> g = make_tile_geo<T>(P);
    constexpr int W = TileWin<T>::W, DEG = TileWin<T>::DEG;
    constexpr int PW = TILE_TS + W - 1;
    const int nt = g.ntx * g.ntx;
    const int nch = 2 * P.nb;
    cx<T>* partI = d.part;
    cx<T>* partR = partI + (size_t)nt * PW * PW;
    cx<T>* partC = partR + (size_t)nt * nch * PW;
    cx<T>* partX = partC + (size_t)nt * nch * PW;
    if (!(flags & GS_SORTED)) {
        // caller-order input: per-point grids differ between problems, so batched
        // launches take sorted input only
        if (!launch_plain()) return hipErrorInvalidValue;
        ProfScope _p(K_ADJ_PREP, s);
        using A = GatherArgs<T>;
        GS_HIP_TRY(launch_site(A{g, u, d.vbuf}, [&](const A& one, const A* many, int count) {
            if (many) hipLaunchKernelGGL((adj_gather_kernel<T, true>), dim3((P.M + 1023) / 1024, count), dim3(256), 0, s, one, many,
                               flags);
        else hipLaunchKernelGGL((adj_gather_kernel<T, false>), dim3((P.M + 1023) / 1024, count), dim3(256), 0, s, one, many,
                               flags);
            return hipGetLastError();
        }));
        u = d.vbuf;
        flags = GS_SORTED;   // gathered and weighted
    }
    // The interior and the column-side/corner kernels read the same staged
    // input and write disjoint partials.  The second runs on the plan's side
    // stream, joined before the merges, in FP64 (the two long FP64 kernels
    // overlap their tails: 8 % per pair) and in FP32 on grids of at most 256
    // tiles, where each kernel alone has one workgroup per CU (the pair of the
    // 262,144-point J = 8 workload: 147 -> 137 us).  On larger FP32 grids each
    // kernel fills the chip and both stay on s, as they do under graph capture.
    hipStream_t s2 = s;
    if constexpr (NB > 0) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        GS_HIP_TRY(hipStreamIsCapturing(s, &cap));
        if ((std::is_same<T, double>::value || nt <= 256) && P.side && cap == hipStreamCaptureStatusNone &&
            launch_plain()) {
            GS_HIP_TRY(hipEventRecord(P.ev_fork, s));
            GS_HIP_TRY(hipStreamWaitEvent(P.side, P.ev_fork, 0));
            s2 = P.side;
        }
        ProfScope _p(K_BND2D, s2);
        using A = AdjArgs<T>;
        GS_HIP_TRY(launch_site(A{g, u, partC, partX}, [&](const A& one, const A* many, int count) {
            // FP32 on grids of more than 256 tiles: the 40 KB stage (four workgroups per CU)
            constexpr int BL4 = std::is_same<T, float>::value ? BND_LDS_FOUR : BND_LDS;
            const dim3 grid(nt, count);
            if (std::is_same<T, float>::value && nt > 256) {
                if (many)
                    hipLaunchKernelGGL((adj_boundary_kernel<T, W, DEG, NB, BL4, true>), grid, dim3(BND_THREADS), 0, s2,
                                       one, many, flags);
                else
                    hipLaunchKernelGGL((adj_boundary_kernel<T, W, DEG, NB, BL4, false>), grid, dim3(BND_THREADS), 0, s2,
                                       one, many, flags);
            } else {
                if (many)
                    hipLaunchKernelGGL((adj_boundary_kernel<T, W, DEG, NB, BND_LDS, true>), grid, dim3(BND_THREADS), 0,
                                       s2, one, many, flags);
                else
                    hipLaunchKernelGGL((adj_boundary_kernel<T, W, DEG, NB, BND_LDS, false>), grid, dim3(BND_THREADS), 0,
                                       s2, one, many, flags);
            }
            return hipGetLastError();
        }));
    }
    {
        ProfScope _p(K_SPREAD2D, s);
        using A = AdjArgs<T>;
        GS_HIP_TRY(launch_site(A{g, u, partI, partR}, [&](const A& one, const A* many, int count) {
            if (many) hipLaunchKernelGGL((adj_interior_kernel<T, W, DEG, NB, true>), dim3(nt, count), dim3(IntShape<W>::THREADS), 0, s,
                               one, many, flags);
        else hipLaunchKernelGGL((adj_interior_kernel<T, W, DEG, NB, false>), dim3(nt, count), dim3(IntShape<W>::THREADS), 0, s,
                               one, many, flags);
            return hipGetLastError();
        }));
    }
    if (s2 != s) {
        GS_HIP_TRY(hipEventRecord(P.ev_join, s2));
        GS_HIP_TRY(hipStreamWaitEvent(s, P.ev_join, 0));
    }
    {
        ProfScope _p(K_MERGE, s);
        const int ngrid = (g.ng * g.ng + 255) / 256;
        if constexpr (NB > 0) {
            const int nside = 2 * nch * (g.ng / 32);
            using A = MergeArgs<T>;
            GS_HIP_TRY(launch_site(A{MergeGridArgs<T>{g, partI, d.grid},
                                     MergeSidesArgs<T>{g, partR, partC, partX, d.sr, d.sc, x}},
                                   [&](const A& one, const A* many, int count) {
                                       const dim3 grid(ngrid + nside + nch * nch, count);
                                       if (many)
                                           hipLaunchKernelGGL((merge_kernel<T, W, true>), grid, dim3(256), 0, s, one,
                                                              many, ngrid, nside);
                                       else
                                           hipLaunchKernelGGL((merge_kernel<T, W, false>), grid, dim3(256), 0, s, one,
                                                              many, ngrid, nside);
                                       return hipGetLastError();
                                   }));
        } else {
            using A = MergeGridArgs<T>;
            GS_HIP_TRY(launch_site(A{g, partI, d.grid}, [&](const A& one, const A* many, int count) {
                if (many)
                    hipLaunchKernelGGL((merge_grid_kernel<T, W, true>), dim3(ngrid, count), dim3(256), 0, s, one, many);
                else
                    hipLaunchKernelGGL((merge_grid_kernel<T, W, false>), dim3(ngrid, count), dim3(256), 0, s, one, many);
                return hipGetLastError();
            }));
        }
    }
    return hipSuccess;
}

template <class T>
hipError_t interp2d_tile(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s, int part) {
    switch (P.nb) {
        case 0: return interp2d_tile_nb<T, 0>(P, x, y, flags, s, part);
        case 2: return interp2d_tile_nb<T, 2>(P, x, y, flags, s, part);
        case 3: return interp2d_tile_nb<T, 3>(P, x, y, flags, s, part);
        case 4: return interp2d_tile_nb<T, 4>(P, x, y, flags, s, part);
        case 5: return interp2d_tile_nb<T, 5>(P, x, y, flags, s, part);
        case 6: return interp2d_tile_nb<T, 6>(P, x, y, flags, s, part);
        case 7: return interp2d_tile_nb<T, 7>(P, x, y, flags, s, part);
        case 8: return interp2d_tile_nb<T, 8>(P, x, y, flags, s, part);
    }
    return hipErrorInvalidValue;
}

template <class T>
hipError_t adjoint2d_tile(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s, const Work<T>& wk) {
    switch (P.nb) {
        case 0: return adjoint2d_tile_nb<T, 0>(P, u, x, flags, s, wk);
        case 2: return adjoint2d_tile_nb<T, 2>(P, u, x, flags, s, wk);
        case 3: return adjoint2d_tile_nb<T, 3>(P, u, x, flags, s, wk);
        case 4: return adjoint2d_tile_nb<T, 4>(P, u, x, flags, s, wk);
        case 5: return adjoint2d_tile_nb<T, 5>(P, u, x, flags, s, wk);
        case 6: return adjoint2d_tile_nb<T, 6>(P, u, x, flags, s, wk);
        case 7: return adjoint2d_tile_nb<T, 7>(P, u, x, flags, s, wk);
        case 8: return adjoint2d_tile_nb<T, 8>(P, u, x, flags, s, wk);
    }
    return hipErrorInvalidValue;
}

template hipError_t interp2d_tile<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t, int);
template hipError_t interp2d_tile<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t, int);
template hipError_t adjoint2d_tile<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t,
                                          const Work<float>&);
template hipError_t adjoint2d_tile<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t,
                                           const Work<double>&);

// partial-buffer elements needed by the 2D adjoint
size_t adjoint2d_part_elems(int ng, int ts, int nb, int w) {
    const size_t nt = (size_t)(ng / ts) * (ng / ts);
    const size_t pw = ts + w - 1;
    return nt * (pw * pw + 2 * (2 * nb) * pw + (2 * nb) * (2 * nb)) + 64;
}

}  // namespace gs
