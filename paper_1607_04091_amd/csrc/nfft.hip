// Matrix-free T and T^H (Sec. 4, Sec. 5, App. C) on gfx950.
//
// Forward  y = T x : interior block D NFFT(x_I) (Sec. 4: I = D F, F x ~ NFFT),
//   boundary blocks L x_L + R x_R (1D); in 2D the nine blocks of
//   eq. 2Dwavelet_border_division: interior by a 2D NFFT, the four sides by
//   1D NFFTs of the boundary rows/columns of X, the four corners densely.
// Adjoint  x = T^H u : the same blocks transposed (App. C, last display).
//
// NFFT (Sec. 3.2, Keiner-Kunis-Potts): oversampling 2, Kaiser-Bessel window
// with W taps per dimension evaluated by per-tap polynomials, deapodization
// by the window's Fourier transform.  Points are kept in cell-sorted order;
// the adjoint spreads by gathering (each grid cell sums the points whose
// window covers it, in a fixed order), so it is deterministic and atomics-free.
#include <algorithm>

#include "common.hpp"
#include "fft.hpp"
#include "prof.hpp"

namespace gs {

// part: 1 = boundary blocks only, 2 = interior (adds the boundary part), 3 = both
template <class T> hipError_t interp2d_tile(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s,
                                            int part = 3);
template <class T> hipError_t adjoint2d_tile(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s,
                                             const Work<T>& wk);
size_t adjoint2d_part_elems(int ng, int ts, int nb, int w);

// ------------------------------------------------------------------ helpers

__device__ inline void decode_pos(uint32_t u, int G, int& cell, float& t) {
    const int sh = 32 - G;
    cell = (int)(u >> sh);
    t = (float)(u & ((1u << sh) - 1u)) * __int_as_float((127 - sh) << 23);
}
__device__ inline void decode_pos(uint64_t u, int G, int& cell, double& t) {
    const int sh = 64 - G;
    cell = (int)(u >> sh);
    t = (double)(u & ((1ull << sh) - 1ull)) * __longlong_as_double((long long)(1023 - sh) << 52);
}

// all W window taps at fractional offset t (tap j at distance t + W/2 - 1 - j)
template <class T, int W, int DEG>
__device__ inline void window_all(T t, const T* __restrict__ coef, T* w) {
    const T x = T(2) * t - T(1);
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T v = coef[j * (DEG + 1) + DEG];
#pragma unroll
        for (int i = DEG - 1; i >= 0; --i) v = v * x + coef[j * (DEG + 1) + i];
        w[j] = v;
    }
}
template <class T, int DEG>
__device__ inline T window_tap(T t, int j, const T* __restrict__ coef) {
    const T x = T(2) * t - T(1);
    const T* c = coef + j * (DEG + 1);
    T v = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) v = v * x + c[i];
    return v;
}

__device__ inline int freq_of(int q, int ng) { return q < (ng >> 1) ? q : q - ng; }

template <class T>
struct Geo {
    int dim, N, nb, ng, G, mask, M;
    int n1, n2, lg1;
    const P_t<T>* pos;
    const cx<T>* chx;
    const cx<T>* chy;
    const T* smu;
    const T* win;
    const T* deap;
    const int32_t* perm;
    const int32_t* cs;
    __device__ int gidx(int l) const { return ((l & (n1 - 1)) * n2) + (l >> lg1); }
    __device__ int bcol(int r) const { return r < nb ? r : N - 1 - (r - nb); }  // boundary channel -> column
    __device__ int bchan(int r) const { return r < nb ? r : r + 1; }            // boundary channel -> chx slot
};

template <class T>
Geo<T> make_geo(const Plan& P) {
    const PrecData<T>& d = prec<T>(P);
    Geo<T> g;
    g.dim = P.dim; g.N = P.N; g.nb = P.nb; g.ng = P.ng; g.G = P.G; g.mask = P.ng - 1; g.M = (int)P.M;
    g.n1 = P.n1; g.n2 = P.n2; g.lg1 = P.lg1;
    g.pos = d.pos; g.chx = d.chx; g.chy = d.chy; g.smu = d.smu; g.win = d.win; g.deap = d.deap;
    g.perm = P.perm; g.cs = P.cell_start;
    return g;
}

// ------------------------------------------------------------------ FFT ops

template <class T> struct OpT2Rows {
    const cx<T>* X; cx<T>* grid; cx<T>* sr; const T* deap; int N, nb, ng;
    __device__ cx<T> load(int i, int q) const {
        const int j = freq_of(q, ng) + (N >> 1);
        if (j < 0 || j >= N) return czero<T>();
        T f = deap[j];
        if (f == T(0)) return czero<T>();
        if (i >= nb && i < N - nb) f *= deap[i];
        return cscale(X[(size_t)i * N + j], f);
    }
    __device__ void store(int i, int q, cx<T> v) const {
        if (i >= nb && i < N - nb) grid[(size_t)((i - (N >> 1)) & (ng - 1)) * ng + q] = v;
        else sr[(size_t)(i < nb ? i : nb + (N - 1 - i)) * ng + q] = v;
    }
};

template <class T> struct OpCols {
    cx<T>* grid; int N, nb, ng, fwd;
    __device__ bool active(int q) const {
        const int k = freq_of(q, ng);
        return k >= -(N >> 1) + nb && k < (N >> 1) - nb;
    }
    __device__ cx<T> load(int col, int q) const {
        if (fwd && !active(q)) return czero<T>();
        return grid[(size_t)q * ng + col];
    }
    __device__ void store(int col, int q, cx<T> v) const {
        if (!fwd && !active(q)) return;
        grid[(size_t)q * ng + col] = v;
    }
};

template <class T> struct OpT2SideCols {
    const cx<T>* X; cx<T>* sc; const T* deap; int N, nb, ng;
    __device__ cx<T> load(int c, int q) const {
        const int i = freq_of(q, ng) + (N >> 1);
        if (i < 0 || i >= N) return czero<T>();
        const T f = deap[i];
        if (f == T(0)) return czero<T>();
        const int j = c < nb ? c : N - 1 - (c - nb);
        return cscale(X[(size_t)i * N + j], f);
    }
    __device__ void store(int c, int q, cx<T> v) const { sc[(size_t)c * ng + q] = v; }
};

// The two adjoint output ops return |stored value|^2 (0 where nothing is
// stored), so that a launch can also sum ||x||^2.  Every entry of x is counted
// once: the row transforms count the interior columns of every row, the
// side-column transforms the boundary columns of the interior rows, and, with
// `corners` set, the row transforms of the boundary rows also count the
// corner entries (boundary row and column), which are final before the row
// pass runs.
template <class T> struct OpTH2Rows {
    const cx<T>* grid; const cx<T>* sr; cx<T>* X; const T* deap; int N, nb, ng;
    int cr1 = 0, cr2 = 0;   // storage order of the grid rows (see Plan::cr1)
    int corners = 0;
    __device__ int row(int k) const { return cr1 ? cr2 * (k & (cr1 - 1)) + k / cr1 : k; }
    __device__ cx<T> load(int i, int q) const {
        if (i >= nb && i < N - nb) return grid[(size_t)row((i - (N >> 1)) & (ng - 1)) * ng + q];
        return sr[(size_t)(i < nb ? i : nb + (N - 1 - i)) * ng + q];
    }
    __device__ double store(int i, int q, cx<T> v) const {
        const int j = freq_of(q, ng) + (N >> 1);
        const bool irow = i >= nb && i < N - nb;
        if (j < nb || j >= N - nb) {
            if (corners && !irow && j >= 0 && j < N) return sq64(X[(size_t)i * N + j]);
            return 0.0;
        }
        T f = deap[j];
        if (irow) f *= deap[i];
        const cx<T> o = cscale(v, f);
        X[(size_t)i * N + j] = o;
        return sq64(o);
    }
};

template <class T> struct OpTH2SideCols {
    const cx<T>* sc; cx<T>* X; const T* deap; int N, nb, ng;
    __device__ cx<T> load(int c, int q) const { return sc[(size_t)c * ng + q]; }
    __device__ double store(int c, int q, cx<T> v) const {
        const int i = freq_of(q, ng) + (N >> 1);
        if (i < nb || i >= N - nb) return 0.0;
        const int j = c < nb ? c : N - 1 - (c - nb);
        const cx<T> o = cscale(v, deap[i]);
        X[(size_t)i * N + j] = o;
        return sq64(o);
    }
};

template <class T> struct Pad1 {
    const cx<T>* x; const T* deap; int N, ng;
    __device__ cx<T> at(int q) const {
        const int j = freq_of(q, ng) + (N >> 1);
        if (j < 0 || j >= N) return czero<T>();
        const T f = deap[j];
        if (f == T(0)) return czero<T>();
        return cscale(x[j], f);
    }
};
template <class T> struct Crop1 {
    cx<T>* x; const T* deap; int N, nb, ng;
    __device__ void put(int q, cx<T> v) const {
        const int j = freq_of(q, ng) + (N >> 1);
        if (j < nb || j >= N - nb) return;
        x[j] = cscale(v, deap[j]);
    }
};
template <class T> struct OpT1Single {
    Pad1<T> in; cx<T>* grid;
    __device__ cx<T> load(int, int q) const { return in.at(q); }
    __device__ void store(int, int q, cx<T> v) const { grid[q] = v; }
};
template <class T> struct OpT1A {   // four-step forward, pass over j1 (columns j2)
    Pad1<T> in; cx<T>* grid; const cx<T>* tw; int n2, ng;
    __device__ cx<T> load(int j2, int j1) const { return in.at(n2 * j1 + j2); }
    __device__ void store(int j2, int k1, cx<T> v) const {
        grid[(size_t)k1 * n2 + j2] = cmul(v, tw[(j2 * k1) & (ng - 1)]);
    }
};
template <class T> struct OpRowsInPlace {  // contiguous rows of length n2
    cx<T>* grid; int n2;
    __device__ cx<T> load(int r, int i) const { return grid[(size_t)r * n2 + i]; }
    __device__ void store(int r, int k, cx<T> v) const { grid[(size_t)r * n2 + k] = v; }
};
template <class T> struct OpTH1Single {
    const cx<T>* grid; Crop1<T> out;
    __device__ cx<T> load(int, int q) const { return grid[q]; }
    __device__ void store(int, int q, cx<T> v) const { out.put(q, v); }
};
template <class T> struct OpTH1P1 {   // four-step adjoint, rows l1, then twiddle
    cx<T>* grid; const cx<T>* tw; int n2, ng;
    __device__ cx<T> load(int l1, int l2) const { return grid[(size_t)l1 * n2 + l2]; }
    __device__ void store(int l1, int k2, cx<T> v) const {
        grid[(size_t)l1 * n2 + k2] = cmul(v, conjc(tw[(l1 * k2) & (ng - 1)]));
    }
};
template <class T> struct OpTH1P2 {   // four-step adjoint, columns k2, crop
    const cx<T>* grid; Crop1<T> out; int n2;
    __device__ cx<T> load(int k2, int l1) const { return grid[(size_t)l1 * n2 + k2]; }
    __device__ void store(int k2, int k1, cx<T> v) const { out.put(n2 * k1 + k2, v); }
};

// ------------------------------------------------------------------ forward interpolation

template <class T, int W, int DEG, int NB>
__global__ void __launch_bounds__(256) interp2d_kernel(Geo<T> g, const cx<T>* __restrict__ grid,
                                                       const cx<T>* __restrict__ sr, const cx<T>* __restrict__ sc,
                                                       const cx<T>* __restrict__ X, cx<T>* __restrict__ y, int flags) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    int cxl, cyl;
    T tx, ty;
    decode_pos(g.pos[m], g.G, cxl, tx);
    decode_pos(g.pos[(size_t)g.M + m], g.G, cyl, ty);
    T wx[W], wy[W];
    window_all<T, W, DEG>(tx, g.win, wx);
    window_all<T, W, DEG>(ty, g.win, wy);
    const int l0x = cxl - W / 2 + 1, l0y = cyl - W / 2 + 1;
    cx<T> I = czero<T>();
#pragma unroll
    for (int a = 0; a < W; ++a) {
        const cx<T>* row = grid + (size_t)((l0x + a) & g.mask) * g.ng;
        cx<T> acc = czero<T>();
#pragma unroll
        for (int b = 0; b < W; ++b) acc = cfma(acc, row[(l0y + b) & g.mask], wy[b]);
        I = cfma(I, acc, wx[a]);
    }
    const size_t M = g.M;
    const cx<T> Dx = g.chx[NB * M + m], Dy = g.chy[NB * M + m];
    cx<T> res = cmul(cmul(Dx, Dy), I);
    if constexpr (NB > 0) {
        cx<T> ay[2 * NB];
#pragma unroll
        for (int r = 0; r < 2 * NB; ++r) ay[r] = g.chy[(size_t)g.bchan(r) * M + m];
#pragma unroll
        for (int r = 0; r < 2 * NB; ++r) {
            const cx<T> ax = g.chx[(size_t)g.bchan(r) * M + m];
            // side x-boundary row r: 1D NFFT along y of row bcol(r) of X
            const cx<T>* s1 = sr + (size_t)r * g.ng;
            cx<T> S = czero<T>();
#pragma unroll
            for (int b = 0; b < W; ++b) S = cfma(S, s1[(l0y + b) & g.mask], wy[b]);
            // corner row r: sum_c ay_c X[bcol(r)][bcol(c)]
            const cx<T>* xr = X + (size_t)g.bcol(r) * g.N;
            cx<T> cr = czero<T>();
#pragma unroll
            for (int c = 0; c < 2 * NB; ++c) cr = cmac(cr, ay[c], xr[g.bcol(c)]);
            res = cmac(res, ax, cadd(cmul(Dy, S), cr));
            // side y-boundary column r: 1D NFFT along x of column bcol(r) of X
            const cx<T>* s2 = sc + (size_t)r * g.ng;
            cx<T> Cc = czero<T>();
#pragma unroll
            for (int a = 0; a < W; ++a) Cc = cfma(Cc, s2[(l0x + a) & g.mask], wx[a]);
            res = cmac(res, cmul(ay[r], Dx), Cc);
        }
    }
    if (flags & GS_WEIGHTED) res = cscale(res, wscale(g.smu[m], flags));
    y[(flags & GS_SORTED) ? m : g.perm[m]] = res;
}

template <class T, int W, int DEG, int NB>
__global__ void __launch_bounds__(256) interp1d_kernel(Geo<T> g, const cx<T>* __restrict__ grid,
                                                       const cx<T>* __restrict__ x, cx<T>* __restrict__ y, int flags) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    int c0;
    T t;
    decode_pos(g.pos[m], g.G, c0, t);
    T w[W];
    window_all<T, W, DEG>(t, g.win, w);
    const int l0 = c0 - W / 2 + 1;
    cx<T> I = czero<T>();
#pragma unroll
    for (int j = 0; j < W; ++j) I = cfma(I, grid[g.gidx((l0 + j) & g.mask)], w[j]);
    const size_t M = g.M;
    cx<T> res = cmul(g.chx[NB * M + m], I);
#pragma unroll
    for (int r = 0; r < 2 * NB; ++r) res = cmac(res, g.chx[(size_t)g.bchan(r) * M + m], x[g.bcol(r)]);
    if (flags & GS_WEIGHTED) res = cscale(res, wscale(g.smu[m], flags));
    y[(flags & GS_SORTED) ? m : g.perm[m]] = res;
}

// ------------------------------------------------------------------ adjoint

// v_m = sqrt(mu)^[weighted] * u[perm m]; vI_m = conj(Dx Dy) v_m (interior value)
template <class T>
__global__ void adj_prep_kernel(Geo<T> g, const cx<T>* __restrict__ u, cx<T>* __restrict__ v,
                                cx<T>* __restrict__ vI, int flags) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    cx<T> val = u[(flags & GS_SORTED) ? m : g.perm[m]];
    if (flags & GS_WEIGHTED) val = cscale(val, wscale(g.smu[m], flags));
    v[m] = val;
    const size_t M = g.M;
    cx<T> D = g.chx[(size_t)g.nb * M + m];
    if (g.dim == 2) D = cmul(D, g.chy[(size_t)g.nb * M + m]);
    vI[m] = cmul(conjc(D), val);
}

// 2D interior spread by gathering: cell (lx, ly) sums every point whose window covers it.
template <class T, int W, int DEG>
__global__ void __launch_bounds__(256) spread2d_kernel(Geo<T> g, const cx<T>* __restrict__ vI, cx<T>* __restrict__ grid) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ng * g.ng) return;
    const int lx = idx >> g.G, ly = idx & g.mask;
    cx<T> acc = czero<T>();
    for (int a = 0; a < W; ++a) {
        const int cxr = (lx - a + W / 2 - 1) & g.mask;
        for (int b = 0; b < W; ++b) {
            const int cy = (ly - b + W / 2 - 1) & g.mask;
            const int cell = (cxr << g.G) | cy;
            const int e = g.cs[cell + 1];
            for (int q = g.cs[cell]; q < e; ++q) {
                int cc;
                T tx, ty;
                decode_pos(g.pos[q], g.G, cc, tx);
                decode_pos(g.pos[(size_t)g.M + q], g.G, cc, ty);
                const T wgt = window_tap<T, DEG>(tx, a, g.win) * window_tap<T, DEG>(ty, b, g.win);
                acc = cfma(acc, vI[q], wgt);
            }
        }
    }
    grid[idx] = acc;
}

// 2D side partials.  Row sides (x-boundary channel r, spread along y over the
// points of one strip of x-cells): value conj(ax_r Dy) v.  Column sides
// (y-boundary channel c, spread along x over one strip of y-cells): conj(ay_c Dx) v.
template <class T, int W, int DEG>
__global__ void __launch_bounds__(256) side_rows_partial_kernel(Geo<T> g, const cx<T>* __restrict__ v,
                                                                cx<T>* __restrict__ part, int strip) {
    const int nch = 2 * g.nb;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nstrip = g.ng / strip;
    if (idx >= nstrip * nch * g.ng) return;
    const int ly = idx % g.ng;
    const int r = (idx / g.ng) % nch;
    const int s = idx / (g.ng * nch);
    const size_t M = g.M;
    const cx<T>* axr = g.chx + (size_t)g.bchan(r) * M;
    const cx<T>* Dy = g.chy + (size_t)g.nb * M;
    cx<T> acc = czero<T>();
    for (int cxr = s * strip; cxr < (s + 1) * strip; ++cxr) {
        for (int b = 0; b < W; ++b) {
            const int cy = (ly - b + W / 2 - 1) & g.mask;
            const int cell = (cxr << g.G) | cy;
            const int e = g.cs[cell + 1];
            for (int q = g.cs[cell]; q < e; ++q) {
                int cc;
                T ty;
                decode_pos(g.pos[M + q], g.G, cc, ty);
                const cx<T> val = cmul(conjc(cmul(axr[q], Dy[q])), v[q]);
                acc = cfma(acc, val, window_tap<T, DEG>(ty, b, g.win));
            }
        }
    }
    part[idx] = acc;
}

template <class T, int W, int DEG>
__global__ void __launch_bounds__(256) side_cols_partial_kernel(Geo<T> g, const cx<T>* __restrict__ v,
                                                                cx<T>* __restrict__ part, int strip) {
    const int nch = 2 * g.nb;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nstrip = g.ng / strip;
    if (idx >= nstrip * nch * g.ng) return;
    const int lx = idx % g.ng;
    const int c = (idx / g.ng) % nch;
    const int s = idx / (g.ng * nch);
    const size_t M = g.M;
    const cx<T>* ayc = g.chy + (size_t)g.bchan(c) * M;
    const cx<T>* Dx = g.chx + (size_t)g.nb * M;
    cx<T> acc = czero<T>();
    for (int a = 0; a < W; ++a) {
        const int cxr = (lx - a + W / 2 - 1) & g.mask;
        const int c0 = (cxr << g.G) | (s * strip);
        const int e = g.cs[c0 + strip];
        for (int q = g.cs[c0]; q < e; ++q) {
            int cc;
            T tx;
            decode_pos(g.pos[q], g.G, cc, tx);
            const cx<T> val = cmul(conjc(cmul(ayc[q], Dx[q])), v[q]);
            acc = cfma(acc, val, window_tap<T, DEG>(tx, a, g.win));
        }
    }
    part[idx] = acc;
}

// out[r*ng + l] = sum_s part[(s*nch + r)*ng + l]  (fixed order)
template <class T>
__global__ void reduce_strips_kernel(const cx<T>* __restrict__ part, cx<T>* __restrict__ out, int nstrip, int count) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    cx<T> acc = czero<T>();
    for (int s = 0; s < nstrip; ++s) acc = cadd(acc, part[(size_t)s * count + idx]);
    out[idx] = acc;
}

// Boundary reductions over points: 2D corners sum_m conj(ax_r ay_c) v_m, 1D
// sum_m conj(a_r) v_m.  One workgroup per chunk of points, one thread lane
// per (r, c) output and 256/npairs point lanes, fixed-order combine.
template <class T>
__global__ void __launch_bounds__(256) boundary_partial_kernel(Geo<T> g, const cx<T>* __restrict__ v,
                                                               cx<T>* __restrict__ part, int chunk) {
    __shared__ cx<T> red[256];
    const int nch = 2 * g.nb;
    const int npairs = g.dim == 2 ? nch * nch : nch;
    const int lanes = 256 / npairs;  // point lanes
    const int pr = threadIdx.x % npairs, pl = threadIdx.x / npairs;
    const size_t M = g.M;
    cx<T> acc = czero<T>();
    if (pl < lanes) {
        const int r = g.dim == 2 ? pr / nch : pr;
        const int c = g.dim == 2 ? pr % nch : 0;
        const cx<T>* ax = g.chx + (size_t)g.bchan(r) * M;
        const cx<T>* ay = g.dim == 2 ? g.chy + (size_t)g.bchan(c) * M : nullptr;
        const int b = blockIdx.x * chunk, e = min(g.M, b + chunk);
        for (int q = b + pl; q < e; q += lanes) {
            cx<T> coef = ax[q];
            if (g.dim == 2) coef = cmul(coef, ay[q]);
            acc = cmacc(acc, coef, v[q]);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < npairs) {
        cx<T> s = czero<T>();
        for (int l = 0; l < lanes; ++l) s = cadd(s, red[l * npairs + threadIdx.x]);
        part[(size_t)blockIdx.x * npairs + threadIdx.x] = s;
    }
}

// One wave per (r, c) output: lane l sums partials l, l + 64, ... in order,
// then a fixed butterfly over the 64 lanes.
template <class T>
__global__ void __launch_bounds__(64) boundary_final_kernel(Geo<T> g, const cx<T>* __restrict__ part, int nblk,
                                                            cx<T>* __restrict__ X) {
    const int nch = 2 * g.nb;
    const int npairs = g.dim == 2 ? nch * nch : nch;
    const int i = blockIdx.x;
    if (i >= npairs) return;
    T sx = T(0), sy = T(0);
    for (int b = threadIdx.x; b < nblk; b += 64) {
        const cx<T> v = part[(size_t)b * npairs + i];
        sx += v.x;
        sy += v.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off);
        sy += __shfl_xor(sy, off);
    }
    if (threadIdx.x != 0) return;
    const cx<T> s = mk<T>(sx, sy);
    if (g.dim == 2) X[(size_t)g.bcol(i / nch) * g.N + g.bcol(i % nch)] = s;
    else X[g.bcol(i)] = s;
}

template <class T, int W, int DEG>
__global__ void __launch_bounds__(256) spread1d_kernel(Geo<T> g, const cx<T>* __restrict__ vI, cx<T>* __restrict__ grid) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= g.ng) return;
    cx<T> acc = czero<T>();
    for (int j = 0; j < W; ++j) {
        const int cell = (l - j + W / 2 - 1) & g.mask;
        const int e = g.cs[cell + 1];
        for (int q = g.cs[cell]; q < e; ++q) {
            int cc;
            T t;
            decode_pos(g.pos[q], g.G, cc, t);
            acc = cfma(acc, vI[q], window_tap<T, DEG>(t, j, g.win));
        }
    }
    grid[g.gidx(l)] = acc;
}

// ------------------------------------------------------------------ launchers

inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }
// workgroups of the boundary-block reduction: about 512 points each, at most
// 256 (the final kernel sums their partials in order)
inline int boundary_blocks(int64_t M) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (M + 511) / 512)); }

template <class T> struct WinParams;
template <> struct WinParams<float> { static constexpr int W = W32, DEG = DEG32; };
template <> struct WinParams<double> { static constexpr int W = W64, DEG = DEG64; };

template <class T, int NB>
hipError_t launch_interp2d(const Plan& P, const Geo<T>& g, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    const PrecData<T>& d = prec<T>(P);
    constexpr int W = WinParams<T>::W, DEG = WinParams<T>::DEG;
    ProfScope _p(K_INTERP2D, s);
    hipLaunchKernelGGL((interp2d_kernel<T, W, DEG, NB>), dim3(nblk(P.M, 256)), dim3(256), 0, s, g, d.grid, d.sr, d.sc,
                       x, y, flags);
    return hipGetLastError();
}
template <class T, int NB>
hipError_t launch_interp1d(const Plan& P, const Geo<T>& g, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    const PrecData<T>& d = prec<T>(P);
    constexpr int W = WinParams<T>::W, DEG = WinParams<T>::DEG;
    ProfScope _p(K_INTERP1D, s);
    hipLaunchKernelGGL((interp1d_kernel<T, W, DEG, NB>), dim3(nblk(P.M, 256)), dim3(256), 0, s, g, d.grid, x, y, flags);
    return hipGetLastError();
}

template <class T>
hipError_t dispatch_interp(const Plan& P, const Geo<T>& g, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    if (P.dim == 2) {
        switch (P.nb) {
            case 0: return launch_interp2d<T, 0>(P, g, x, y, flags, s);
            case 2: return launch_interp2d<T, 2>(P, g, x, y, flags, s);
            case 3: return launch_interp2d<T, 3>(P, g, x, y, flags, s);
            case 4: return launch_interp2d<T, 4>(P, g, x, y, flags, s);
            case 5: return launch_interp2d<T, 5>(P, g, x, y, flags, s);
            case 6: return launch_interp2d<T, 6>(P, g, x, y, flags, s);
            case 7: return launch_interp2d<T, 7>(P, g, x, y, flags, s);
            case 8: return launch_interp2d<T, 8>(P, g, x, y, flags, s);
        }
    } else {
        switch (P.nb) {
            case 0: return launch_interp1d<T, 0>(P, g, x, y, flags, s);
            case 2: return launch_interp1d<T, 2>(P, g, x, y, flags, s);
            case 3: return launch_interp1d<T, 3>(P, g, x, y, flags, s);
            case 4: return launch_interp1d<T, 4>(P, g, x, y, flags, s);
            case 5: return launch_interp1d<T, 5>(P, g, x, y, flags, s);
            case 6: return launch_interp1d<T, 6>(P, g, x, y, flags, s);
            case 7: return launch_interp1d<T, 7>(P, g, x, y, flags, s);
            case 8: return launch_interp1d<T, 8>(P, g, x, y, flags, s);
        }
    }
    return hipErrorInvalidValue;
}

#define GS_TIMED(id, ...)          \
    do {                           \
        ProfScope _p((id), s);     \
        __VA_ARGS__;               \
    } while (0)

int norm_parts_TH(const Plan& P) { return P.dim == 2 && P.ts == TILE ? P.N + 2 * P.nb : 0; }

template <class T>
hipError_t launch_apply_T(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    const PrecData<T>& d = prec<T>(P);
    const Geo<T> g = make_geo<T>(P);
    const int N = P.N, nb = P.nb, ng = P.ng;
    const bool tiled = P.dim == 2 && P.ts == TILE;
    if (P.dim == 2) {
        const OpT2Rows<T> rows{x, d.grid, d.sr, d.deap, N, nb, ng};
        if (nb) {
            // the 2nb side-column transforms share the row launch
            using J = OpJoin<T, OpT2Rows<T>, OpT2SideCols<T>>;
            GS_TIMED(K_FFT_ROWS_T, GS_HIP_TRY((launch_fft<T, -1>(J{rows, OpT2SideCols<T>{x, d.sc, d.deap, N, nb, ng}, N},
                                                               N + 2 * nb, ng, 1, d.tw, ng, s))));
        } else {
            GS_TIMED(K_FFT_ROWS_T, GS_HIP_TRY((launch_fft<T, -1>(rows, N, ng, 1, d.tw, ng, s))));
        }
        if (P.cr1) {
            auto mk = [&](int L) { return GridLoad<T>{d.grid, L, N, nb, 1}; };
            GS_TIMED(K_FFT_COLS_T, GS_HIP_TRY((launch_colfft_split<T, -1>(P.cr1, ng, mk, d.grid, d.tw, N, nb, 0, s))));
        } else {
            GS_TIMED(K_FFT_COLS_T, GS_HIP_TRY((launch_fft<T, -1>(OpCols<T>{d.grid, N, nb, ng, 1}, ng, ng,
                                                               col_batch<T>(ng), d.tw, ng, s))));
        }
    } else {
        const Pad1<T> pad{x, d.deap, N, ng};
        if (ng <= FFT_MAX_LDS) {
            GS_TIMED(K_FFT1_T, GS_HIP_TRY((launch_fft<T, -1>(OpT1Single<T>{pad, d.grid}, 1, ng, 1, d.tw, ng, s))));
        } else {
            GS_TIMED(K_FFT1_T, GS_HIP_TRY((launch_fft<T, -1>(OpT1A<T>{pad, d.grid, d.tw, P.n2, ng}, P.n2, P.n1,
                                                           col_batch<T>(P.n1), d.tw, ng, s))));
            GS_TIMED(K_FFT1_T, GS_HIP_TRY((launch_fft<T, -1>(OpRowsInPlace<T>{d.grid, P.n2}, P.n1, P.n2, 1, d.tw,
                                                           ng, s))));
        }
    }
    if (tiled) return interp2d_tile<T>(P, x, y, flags, s);
    return dispatch_interp<T>(P, g, x, y, flags, s);
}

template <class T>
hipError_t launch_apply_TH(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s, const Work<T>* work,
                           double* nsq) {
    const PrecData<T>& d = prec<T>(P);
    const Work<T> wk = work ? *work : plan_work(d);
    const Geo<T> g = make_geo<T>(P);
    constexpr int W = WinParams<T>::W, DEG = WinParams<T>::DEG;
    const int N = P.N, nb = P.nb, ng = P.ng;
    if (P.dim == 2 && P.ts == TILE) {
        GS_HIP_TRY(adjoint2d_tile<T>(P, u, x, flags, s, wk));
        if (P.cr1) {
            auto mk = [&](int L) { return GridLoad<T>{wk.grid, L, N, nb, 0}; };
            GS_TIMED(K_FFT_COLS_TH, GS_HIP_TRY((launch_colfft_split<T, +1>(P.cr1, ng, mk, wk.grid, d.tw, N, nb, 1, s))));
        } else {
            GS_TIMED(K_FFT_COLS_TH, GS_HIP_TRY((launch_fft<T, +1>(OpCols<T>{wk.grid, N, nb, ng, 0}, ng, ng,
                                                                col_batch<T>(ng), d.tw, ng, s))));
        }
        OpTH2Rows<T> rows{wk.grid, wk.sr, x, d.deap, N, nb, ng, P.cr1, P.cr2};
        rows.corners = nsq != nullptr;
        if (nb) {
            using J = OpJoin<T, OpTH2Rows<T>, OpTH2SideCols<T>>;
            GS_TIMED(K_FFT_ROWS_TH, GS_HIP_TRY((launch_fft<T, +1>(J{rows, OpTH2SideCols<T>{wk.sc, x, d.deap, N, nb, ng}, N},
                                                                N + 2 * nb, ng, 1, d.tw, ng, s, nsq))));
        } else {
            GS_TIMED(K_FFT_ROWS_TH, GS_HIP_TRY((launch_fft<T, +1>(rows, N, ng, 1, d.tw, ng, s, nsq))));
        }
        return hipSuccess;
    }
    cx<T>* v = wk.vbuf;
    cx<T>* vI = wk.part;  // first M entries of the partial buffer
    cx<T>* part = wk.part + P.M;
    GS_TIMED(K_ADJ_PREP, hipLaunchKernelGGL((adj_prep_kernel<T>), dim3(nblk(P.M, 256)), dim3(256), 0, s, g, u, v, vI,
                                            flags));
    GS_HIP_TRY(hipGetLastError());
    const int nbl = boundary_blocks(P.M);
    if (nb) {
        GS_TIMED(K_BOUNDARY_PARTIAL, hipLaunchKernelGGL((boundary_partial_kernel<T>), dim3(nbl), dim3(256), 0, s, g, v,
                                                        part, (int)((P.M + nbl - 1) / nbl)));
        GS_HIP_TRY(hipGetLastError());
        GS_TIMED(K_BOUNDARY_FINAL,
                 hipLaunchKernelGGL((boundary_final_kernel<T>), dim3(P.dim == 2 ? 4 * nb * nb : 2 * nb), dim3(64), 0, s,
                                    g, part, nbl, x));
        GS_HIP_TRY(hipGetLastError());
    }
    if (P.dim == 2) {
        GS_TIMED(K_SPREAD2D, hipLaunchKernelGGL((spread2d_kernel<T, W, DEG>), dim3(nblk((int64_t)ng * ng, 256)),
                                                dim3(256), 0, s, g, vI, wk.grid));
        GS_HIP_TRY(hipGetLastError());
        if (nb) {
            const int strip = std::min(ng, 64);
            const int nstrip = ng / strip;
            const int count = 2 * nb * ng;
            GS_TIMED(K_SIDE_ROWS, hipLaunchKernelGGL((side_rows_partial_kernel<T, W, DEG>),
                                                     dim3(nblk((int64_t)nstrip * count, 256)), dim3(256), 0, s, g, v,
                                                     part, strip));
            GS_HIP_TRY(hipGetLastError());
            GS_TIMED(K_REDUCE_STRIPS, hipLaunchKernelGGL((reduce_strips_kernel<T>), dim3(nblk(count, 256)), dim3(256),
                                                         0, s, part, wk.sr, nstrip, count));
            GS_HIP_TRY(hipGetLastError());
            GS_TIMED(K_SIDE_COLS, hipLaunchKernelGGL((side_cols_partial_kernel<T, W, DEG>),
                                                     dim3(nblk((int64_t)nstrip * count, 256)), dim3(256), 0, s, g, v,
                                                     part, strip));
            GS_HIP_TRY(hipGetLastError());
            GS_TIMED(K_REDUCE_STRIPS, hipLaunchKernelGGL((reduce_strips_kernel<T>), dim3(nblk(count, 256)), dim3(256),
                                                         0, s, part, wk.sc, nstrip, count));
            GS_HIP_TRY(hipGetLastError());
        }
        GS_TIMED(K_FFT_COLS_TH, GS_HIP_TRY((launch_fft<T, +1>(OpCols<T>{wk.grid, N, nb, ng, 0}, ng, ng,
                                                            col_batch<T>(ng), d.tw, ng, s))));
        GS_TIMED(K_FFT_ROWS_TH, GS_HIP_TRY((launch_fft<T, +1>(OpTH2Rows<T>{wk.grid, wk.sr, x, d.deap, N, nb, ng}, N, ng,
                                                            1, d.tw, ng, s))));
        if (nb)
            GS_TIMED(K_FFT_SIDECOLS_TH,
                     GS_HIP_TRY((launch_fft<T, +1>(OpTH2SideCols<T>{wk.sc, x, d.deap, N, nb, ng}, 2 * nb, ng,
                                                   1, d.tw, ng, s))));
    } else {
        GS_TIMED(K_SPREAD1D, hipLaunchKernelGGL((spread1d_kernel<T, W, DEG>), dim3(nblk(ng, 256)), dim3(256), 0, s, g,
                                                vI, wk.grid));
        GS_HIP_TRY(hipGetLastError());
        const Crop1<T> crop{x, d.deap, N, nb, ng};
        if (ng <= FFT_MAX_LDS) {
            GS_TIMED(K_FFT1_TH, GS_HIP_TRY((launch_fft<T, +1>(OpTH1Single<T>{wk.grid, crop}, 1, ng, 1, d.tw, ng, s))));
        } else {
            GS_TIMED(K_FFT1_TH, GS_HIP_TRY((launch_fft<T, +1>(OpTH1P1<T>{wk.grid, d.tw, P.n2, ng}, P.n1, P.n2, 1, d.tw,
                                                            ng, s))));
            GS_TIMED(K_FFT1_TH, GS_HIP_TRY((launch_fft<T, +1>(OpTH1P2<T>{wk.grid, crop, P.n2}, P.n2, P.n1,
                                                            col_batch<T>(P.n1), d.tw, ng, s))));
        }
    }
    return hipSuccess;
}

template hipError_t launch_apply_T<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t);
template hipError_t launch_apply_T<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t);
template hipError_t launch_apply_TH<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t,
                                           const Work<float>*, double*);
template hipError_t launch_apply_TH<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t,
                                            const Work<double>*, double*);

// partial-buffer size needed by the adjoint (elements)
size_t adjoint_part_elems(int dim, int64_t M, int nb, int ng) {
    size_t need = (size_t)M;  // vI
    size_t b = (size_t)boundary_blocks(M) * (size_t)(dim == 2 ? 4 * nb * nb : 2 * nb);
    size_t sides = 0;
    if (dim == 2 && nb) {
        const int strip = std::min(ng, 64);
        sides = (size_t)(ng / strip) * 2 * nb * ng;
    }
    size_t v1 = need + std::max(b, sides) + 64;
    if (dim == 2) {
        const int ts = std::min(TILE, ng);
        v1 = std::max(v1, adjoint2d_part_elems(ng, ts, nb, std::max(W32, W64)));
    }
    return v1;
}

}  // namespace gs
