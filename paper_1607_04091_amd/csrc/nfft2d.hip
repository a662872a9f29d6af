// 2D T and T^H with tile-staged kernels (Sec. 5, App. C; NFFT of Sec. 3.2).
//
// Points are sorted tile-major (tiles of TS x TS grid cells, row-major cells
// inside a tile), so the points of a tile are contiguous.
//
// Forward (interp_tile_kernel): one workgroup per tile stages the grid
// window it needs (TS+W-1 squared), the matching segments of the 1D side
// grids and the corner block of X in LDS; each thread then evaluates one
// point: interior 2D interpolation, the four side blocks (1D interpolation
// of the boundary rows/columns), the four corner blocks, the scales
// D_x D_y, boundary channels and sqrt(mu).
//
// Adjoint (adjoint_tile_kernel): one workgroup per tile owns the points of
// the tile.  Per chunk of points it stages, once per point, the window taps
// and the channel products in LDS; then
//   * column-owner threads (one per padded output column and block of cell
//     rows) gather the interior 2D spread into register accumulators for the
//     W+RB-1 output rows that block touches, plus the row-side (x-boundary)
//     channels;
//   * row-owner threads gather the column-side (y-boundary) channels;
//   * one wavefront accumulates the corner blocks sum_m conj(ax_r ay_c) v_m
//     as a matrix product with MFMA.
// The tile writes its partial padded grid, side and corner sums; a merge
// kernel adds the partials of neighbouring tiles in a fixed order.  No
// atomics are used, and results are bitwise reproducible.
#include <algorithm>

#include "common.hpp"
#include "prof.hpp"

namespace gs {

template <class T>
struct TileGeo {
    int N, nb, ng, G, mask, M, ts, lts, ntx;
    const P_t<T>* pos;
    const cx<T>* chx;
    const cx<T>* chy;
    const T* smu;
    const T* win;
    const int32_t* perm;
    const int32_t* cs;
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

template <class T, int W, int DEG>
__device__ inline void taps_all(T t, const T* __restrict__ coef, T* w) {
    const T x = T(2) * t - T(1);
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T v = coef[j * (DEG + 1) + DEG];
#pragma unroll
        for (int i = DEG - 1; i >= 0; --i) v = v * x + coef[j * (DEG + 1) + i];
        w[j] = v;
    }
}

constexpr int TILE_TS = 32;     // grid cells per tile side
constexpr int TILE_RB = 8;      // cell rows per column-owner block

// ------------------------------------------------------------------ forward

template <class T, int W, int DEG, int NB>
__global__ void __launch_bounds__(256) interp_tile_kernel(TileGeo<T> g, const cx<T>* __restrict__ grid,
                                                          const cx<T>* __restrict__ sr, const cx<T>* __restrict__ sc,
                                                          const cx<T>* __restrict__ X, cx<T>* __restrict__ y,
                                                          int flags) {
    constexpr int TS = TILE_TS, PW = TS + W - 1, NCH = 2 * NB;
    __shared__ cx<T> sG[PW * PW];
    __shared__ cx<T> sSR[NCH > 0 ? NCH * PW : 1];
    __shared__ cx<T> sSC[NCH > 0 ? NCH * PW : 1];
    __shared__ cx<T> sXC[NCH > 0 ? NCH * NCH : 1];
    const int tile = blockIdx.x;
    const int q0 = g.cs[tile << (2 * g.lts)];
    const int q1 = g.cs[(tile + 1) << (2 * g.lts)];
    if (q0 == q1) return;
    const int t0x = (tile / g.ntx) << g.lts, t0y = (tile % g.ntx) << g.lts;
    const int ox = t0x - (W / 2 - 1), oy = t0y - (W / 2 - 1);
    for (int e = threadIdx.x; e < PW * PW; e += blockDim.x) {
        const int i = e / PW, j = e - i * PW;
        sG[e] = grid[(size_t)((ox + i) & g.mask) * g.ng + ((oy + j) & g.mask)];
    }
    if constexpr (NB > 0) {
        for (int e = threadIdx.x; e < NCH * PW; e += blockDim.x) {
            const int r = e / PW, j = e - r * PW;
            sSR[e] = sr[(size_t)r * g.ng + ((oy + j) & g.mask)];
            sSC[e] = sc[(size_t)r * g.ng + ((ox + j) & g.mask)];
        }
        for (int e = threadIdx.x; e < NCH * NCH; e += blockDim.x) {
            const int r = e / NCH, c = e - r * NCH;
            sXC[e] = X[(size_t)g.bcol(r) * g.N + g.bcol(c)];
        }
    }
    __syncthreads();
    const size_t M = g.M;
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
        const cx<T> Dx = g.chx[NB * M + q], Dy = g.chy[NB * M + q];
        cx<T> res = cmul(cmul(Dx, Dy), I);
        if constexpr (NB > 0) {
            cx<T> ay[NCH];
#pragma unroll
            for (int r = 0; r < NCH; ++r) ay[r] = g.chy[(size_t)(r < NB ? r : r + 1) * M + q];
#pragma unroll
            for (int r = 0; r < NCH; ++r) {
                const cx<T> ax = g.chx[(size_t)(r < NB ? r : r + 1) * M + q];
                cx<T> S = czero<T>();
#pragma unroll
                for (int b = 0; b < W; ++b) S = cfma(S, sSR[r * PW + ly + b], wy[b]);
                cx<T> cr = czero<T>();
#pragma unroll
                for (int c = 0; c < NCH; ++c) cr = cmac(cr, ay[c], sXC[r * NCH + c]);
                res = cmac(res, ax, cadd(cmul(Dy, S), cr));
                cx<T> Cc = czero<T>();
#pragma unroll
                for (int a = 0; a < W; ++a) Cc = cfma(Cc, sSC[r * PW + lx + a], wx[a]);
                res = cmac(res, cmul(ay[r], Dx), Cc);
            }
        }
        if (flags & GS_WEIGHTED) res = cscale(res, g.smu[q]);
        y[(flags & GS_SORTED) ? q : g.perm[q]] = res;
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

template <class T, int W, int NB, int CH>
struct AdjLDS {
    static constexpr int TS = TILE_TS, PW = TS + W - 1, NCH = 2 * NB, NRB = TS / TILE_RB;
    static constexpr int NE = NB > 0 ? 4 * NB : 1;              // real entries of e (re/im of 2NB channels)
    static constexpr int NBLK = (4 * NB + 15) / 16;              // 16x16 MFMA blocks per side
    // staging
    // column-side aggregation: thread (row, channel group), CPT channels each
    static constexpr int CPT = NCH > 0 ? (NCH + 3) / 4 : 1;
    static constexpr int NCP = NCH > 0 ? (NCH + CPT - 1) / CPT : 0;
    // point index fastest for the arrays the gathering threads read
    struct Stage {
        int cy[CH];
        cx<T> v[CH];
        T wx[W][CH];
        T wy[W][CH];
        cx<T> cr[NCH > 0 ? NCH : 1][CH];
        cx<T> dc[NCH > 0 ? NCH : 1][CH];
        T e[CH][NE];
        T f[CH][NE];
    };
    struct Out {
        cx<T> P[PW][PW];
        cx<T> PR[NCH > 0 ? NCH : 1][PW];
        cx<T> PC[NCH > 0 ? NCH : 1][PW];
    };
    static constexpr size_t bytes = sizeof(Stage) > sizeof(Out) ? sizeof(Stage) : sizeof(Out);
};

template <class T, int W, int DEG, int NB, int CH>
__global__ void __launch_bounds__(384) adjoint_tile_kernel(TileGeo<T> g, const cx<T>* __restrict__ u, int flags,
                                                           cx<T>* __restrict__ partI, cx<T>* __restrict__ partR,
                                                           cx<T>* __restrict__ partC, cx<T>* __restrict__ partX) {
    using L = AdjLDS<T, W, NB, CH>;
    constexpr int TS = TILE_TS, RB = TILE_RB, PW = L::PW, NCH = L::NCH, NRB = L::NRB, NE = L::NE;
    constexpr int NACC = RB + W - 1;
    constexpr int NA = PW * NRB;                  // column-owner threads
    constexpr int CPT = L::CPT, NCP = L::NCP;
    constexpr int NBT = NB > 0 ? TS * NCP : 0;    // row-aggregation threads (row, channel group)
    __shared__ int off[TS * TS + 1];
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[L::bytes];
    __shared__ T cbuf[NB > 0 ? L::NBLK * L::NBLK * 256 : 1];
    typename L::Stage& S = *reinterpret_cast<typename L::Stage*>(lds_raw);

    const int tile = blockIdx.x;
    const int tid = threadIdx.x;
    const int kbase = tile << (2 * g.lts);
    const int q0 = g.cs[kbase];
    const int cnt = g.cs[kbase + TS * TS] - q0;
    const int t0y = (tile % g.ntx) << g.lts;
    for (int c = tid; c <= TS * TS; c += blockDim.x) off[c] = g.cs[kbase + c] - q0;
    const size_t M = g.M;

    // role A: (ply, rb); role B: (plx, half); role C: last wavefront (corners)
    const bool roleA = tid < NA;
    const int ply = tid % PW, rb = tid / PW;
    const bool roleB = NB > 0 && tid >= NA && tid < NA + NBT;
    const int brow = (tid - NA) / (NCP > 0 ? NCP : 1), bcg = (tid - NA) % (NCP > 0 ? NCP : 1);
    const int wave = tid >> 6, lane = tid & 63;
    const bool roleC = NB > 0 && wave == (int)(blockDim.x >> 6) - 1;

    cx<T> accI[NACC];
    cx<T> accR[NCH > 0 ? NCH : 1];
    cx<T> accB[CPT][W];
#pragma unroll
    for (int i = 0; i < NACC; ++i) accI[i] = czero<T>();
#pragma unroll
    for (int i = 0; i < (NCH > 0 ? NCH : 1); ++i) accR[i] = czero<T>();
#pragma unroll
    for (int i = 0; i < CPT; ++i)
#pragma unroll
        for (int a = 0; a < W; ++a) accB[i][a] = czero<T>();
    typename Mfma<T>::acc accM[L::NBLK * L::NBLK > 0 ? L::NBLK * L::NBLK : 1];
#pragma unroll
    for (int i = 0; i < (L::NBLK * L::NBLK > 0 ? L::NBLK * L::NBLK : 1); ++i) accM[i] = Mfma<T>::zero();

    for (int c0 = 0; c0 < cnt; c0 += CH) {
        const int c1 = min(cnt, c0 + CH);
        __syncthreads();
        // ---- stage: three tasks per point spread over the workgroup
        for (int job = tid; job < 3 * CH; job += blockDim.x) {
            const int t = job % CH, task = job / CH;
            if (c0 + t >= c1) continue;
            const int q = q0 + c0 + t;
            cx<T> v = u[(flags & GS_SORTED) ? q : g.perm[q]];
            if (flags & GS_WEIGHTED) v = cscale(v, g.smu[q]);
            const cx<T> Dx = g.chx[NB * M + q], Dy = g.chy[NB * M + q];
            if (task == 0) {
                int cxg, cyg;
                T tx, ty;
                decode_pos2(g.pos[q], g.G, cxg, tx);
                decode_pos2(g.pos[M + q], g.G, cyg, ty);
                S.cy[t] = cyg - t0y;
                S.v[t] = cmul(conjc(cmul(Dx, Dy)), v);
                T w[W];
                taps_all<T, W, DEG>(tx, g.win, w);
#pragma unroll
                for (int j = 0; j < W; ++j) S.wx[j][t] = w[j];
                taps_all<T, W, DEG>(ty, g.win, w);
#pragma unroll
                for (int j = 0; j < W; ++j) S.wy[j][t] = w[j];
            } else if constexpr (NB > 0) {
                if (task == 1) {
#pragma unroll
                    for (int r = 0; r < NCH; ++r) {
                        const cx<T> ax = g.chx[(size_t)(r < NB ? r : r + 1) * M + q];
                        S.cr[r][t] = cmul(conjc(cmul(ax, Dy)), v);
                        const cx<T> e = cmul(conjc(ax), v);
                        S.e[t][r] = e.x;
                        S.e[t][NCH + r] = e.y;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NCH; ++r) {
                        const cx<T> ay = g.chy[(size_t)(r < NB ? r : r + 1) * M + q];
                        S.dc[r][t] = cmul(conjc(cmul(ay, Dx)), v);
                        S.f[t][r] = ay.x;
                        S.f[t][NCH + r] = -ay.y;
                    }
                }
            }
        }
        __syncthreads();
        if (roleA) {
            const int cy_lo = max(0, ply - (W - 1)), cy_hi = min(TS - 1, ply);
            if (cy_lo <= cy_hi) {
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    const int cxl = rb * RB + rr;
                    const int pa = max(off[cxl * TS + cy_lo], c0), pb = min(off[cxl * TS + cy_hi + 1], c1);
                    for (int p = pa; p < pb; ++p) {
                        const int t = p - c0;
                        const int b = ply - S.cy[t];
                        const T wyb = S.wy[b][t];
                        const cx<T> tv = cscale(S.v[t], wyb);
#pragma unroll
                        for (int a = 0; a < W; ++a) accI[rr + a] = cfma(accI[rr + a], tv, S.wx[a][t]);
                        if constexpr (NB > 0) {
#pragma unroll
                            for (int r = 0; r < NCH; ++r) accR[r] = cfma(accR[r], S.cr[r][t], wyb);
                        }
                    }
                }
            }
        } else if (roleB) {
            if constexpr (NB > 0) {
                // R[row][c][a] += d_c(m) wx_m[a] over the row's points (all lanes of a row read one point)
                const int pa = max(off[brow * TS], c0), pb = min(off[brow * TS + TS], c1);
                for (int p = pa; p < pb; ++p) {
                    const int t = p - c0;
                    T w[W];
#pragma unroll
                    for (int a = 0; a < W; ++a) w[a] = S.wx[a][t];
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        const int c = bcg * CPT + k;
                        if (c < NCH) {
                            const cx<T> dv = S.dc[c][t];
#pragma unroll
                            for (int a = 0; a < W; ++a) accB[k][a] = cfma(accB[k][a], dv, w[a]);
                        }
                    }
                }
            }
        } else if (roleC) {
            if constexpr (NB > 0) {
                const int i = lane & 15, kk = lane >> 4;
                for (int k4 = c0; k4 < c1; k4 += 4) {
                    const int p = k4 + kk;
                    const bool ok = p < c1;
#pragma unroll
                    for (int bi = 0; bi < L::NBLK; ++bi) {
                        const int ie = bi * 16 + i;
                        const T av = (ok && ie < NE) ? S.e[p - c0][ie] : T(0);
#pragma unroll
                        for (int bj = 0; bj < L::NBLK; ++bj) {
                            const int jf = bj * 16 + i;
                            const T bv = (ok && jf < NE) ? S.f[p - c0][jf] : T(0);
                            accM[bi * L::NBLK + bj] = Mfma<T>::step(av, bv, accM[bi * L::NBLK + bj]);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // ---- combine the row blocks into the padded partial, one block per round (fixed order)
    typename L::Out& O = *reinterpret_cast<typename L::Out*>(lds_raw);
    for (int e = tid; e < PW * PW; e += blockDim.x) (&O.P[0][0])[e] = czero<T>();
    if constexpr (NB > 0) {
        for (int e = tid; e < NCH * PW; e += blockDim.x) (&O.PR[0][0])[e] = czero<T>();
        for (int e = tid; e < NCH * PW; e += blockDim.x) (&O.PC[0][0])[e] = czero<T>();
    }
    __syncthreads();
    if constexpr (NB > 0) {
        // column sides: C_c[plx] = sum_a R[plx - a][c][a]; rows with equal residue mod W
        // touch disjoint outputs, so W rounds fold them without conflicts (fixed order)
        for (int k = 0; k < W; ++k) {
            if (roleB && brow % W == k) {
#pragma unroll
                for (int kk = 0; kk < CPT; ++kk) {
                    const int c = bcg * CPT + kk;
                    if (c < NCH) {
#pragma unroll
                        for (int a = 0; a < W; ++a) O.PC[c][brow + a] = cadd(O.PC[c][brow + a], accB[kk][a]);
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int b = 0; b < NRB; ++b) {
        if (roleA && rb == b) {
#pragma unroll
            for (int i = 0; i < NACC; ++i) O.P[b * RB + i][ply] = cadd(O.P[b * RB + i][ply], accI[i]);
            if constexpr (NB > 0) {
#pragma unroll
                for (int r = 0; r < NCH; ++r) O.PR[r][ply] = cadd(O.PR[r][ply], accR[r]);
            }
        }
        __syncthreads();
    }
    cx<T>* pI = partI + (size_t)tile * PW * PW;
    for (int e = tid; e < PW * PW; e += blockDim.x) pI[e] = (&O.P[0][0])[e];
    if constexpr (NB > 0) {
        cx<T>* pR = partR + (size_t)tile * NCH * PW;
        for (int e = tid; e < NCH * PW; e += blockDim.x) pR[e] = (&O.PR[0][0])[e];
        cx<T>* pC = partC + (size_t)tile * NCH * PW;
        for (int e = tid; e < NCH * PW; e += blockDim.x) pC[e] = (&O.PC[0][0])[e];
        if (roleC) {
            // lane holds four rows of column lane%16 of each 16x16 block
#pragma unroll
            for (int bi = 0; bi < L::NBLK; ++bi)
#pragma unroll
                for (int bj = 0; bj < L::NBLK; ++bj)
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv) {
                        const int row = bi * 16 + Mfma<T>::row(lane, vv), col = bj * 16 + (lane & 15);
                        cbuf[row * (16 * L::NBLK) + col] = accM[bi * L::NBLK + bj][vv];
                    }
        }
        __syncthreads();
        cx<T>* pX = partX + (size_t)tile * NCH * NCH;
        constexpr int LD = 16 * L::NBLK;
        for (int e = tid; e < NCH * NCH; e += blockDim.x) {
            const int r = e / NCH, c = e - r * NCH;
            const T re = cbuf[r * LD + c] - cbuf[(NCH + r) * LD + NCH + c];
            const T im = cbuf[r * LD + NCH + c] + cbuf[(NCH + r) * LD + c];
            pX[e] = mk<T>(re, im);
        }
    }
}

// grid cell (gx, gy) = sum of the padded tile partials that cover it (fixed order)
template <class T, int W>
__global__ void merge_grid_kernel(TileGeo<T> g, const cx<T>* __restrict__ partI, cx<T>* __restrict__ grid) {
    constexpr int TS = TILE_TS, PW = TS + W - 1, H = W / 2 - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
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

// side grids: sr[r][gy] sums over every tile row tx, sc[c][gx] over every tile column ty
template <class T, int W>
__global__ void merge_sides_kernel(TileGeo<T> g, const cx<T>* __restrict__ partR, const cx<T>* __restrict__ partC,
                                   cx<T>* __restrict__ sr, cx<T>* __restrict__ sc) {
    constexpr int TS = TILE_TS, PW = TS + W - 1, H = W / 2 - 1;
    const int nch = 2 * g.nb;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * nch * g.ng) return;
    const int which = idx / (nch * g.ng);
    const int r = (idx / g.ng) % nch, gl = idx % g.ng;
    const int sl = (gl + H) & g.mask;
    const int t0 = sl >> g.lts, p0 = sl & (TS - 1);
    const bool o = p0 < W - 1;
    const int tm = (t0 + g.ntx - 1) % g.ntx;
    cx<T> s = czero<T>();
    if (which == 0) {   // row sides: tiles (t, t0) and (t, tm) for all t
        for (int t = 0; t < g.ntx; ++t) {
            if (o) s = cadd(s, partR[((size_t)(t * g.ntx + tm) * nch + r) * PW + p0 + TS]);
            s = cadd(s, partR[((size_t)(t * g.ntx + t0) * nch + r) * PW + p0]);
        }
        sr[(size_t)r * g.ng + gl] = s;
    } else {            // column sides: tiles (t0, t) and (tm, t)
        for (int t = 0; t < g.ntx; ++t) {
            if (o) s = cadd(s, partC[((size_t)(tm * g.ntx + t) * nch + r) * PW + p0 + TS]);
            s = cadd(s, partC[((size_t)(t0 * g.ntx + t) * nch + r) * PW + p0]);
        }
        sc[(size_t)r * g.ng + gl] = s;
    }
}

// corners: X[bcol(r)][bcol(c)] = sum over all tiles (fixed tree order)
template <class T>
__global__ void __launch_bounds__(256) merge_corners_kernel(TileGeo<T> g, const cx<T>* __restrict__ partX, int ntiles,
                                                            cx<T>* __restrict__ X) {
    __shared__ cx<T> sh[256];
    const int nch = 2 * g.nb;
    const int e = blockIdx.x;       // (r, c)
    cx<T> s = czero<T>();
    for (int t = threadIdx.x; t < ntiles; t += 256) s = cadd(s, partX[(size_t)t * nch * nch + e]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] = cadd(sh[threadIdx.x], sh[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) X[(size_t)g.bcol(e / nch) * g.N + g.bcol(e % nch)] = sh[0];
}

// ------------------------------------------------------------------ launchers

template <class T>
TileGeo<T> make_tile_geo(const Plan& P) {
    const PrecData<T>& d = prec<T>(P);
    TileGeo<T> g;
    g.N = P.N; g.nb = P.nb; g.ng = P.ng; g.G = P.G; g.mask = P.ng - 1; g.M = (int)P.M;
    g.ts = P.ts; g.lts = ilog2(P.ts); g.ntx = P.ng / P.ts;
    g.pos = d.pos; g.chx = d.chx; g.chy = d.chy; g.smu = d.smu; g.win = d.win;
    g.perm = P.perm; g.cs = P.cell_start;
    return g;
}

template <class T> struct TileWin;
template <> struct TileWin<float> { static constexpr int W = W32, DEG = DEG32, CH = 128; };
template <> struct TileWin<double> { static constexpr int W = W64, DEG = DEG64, CH = 64; };
// staging chunk: points per LDS refill (smaller for many boundary channels)
template <class T, int NB> constexpr int tile_chunk() { return NB > 4 ? TileWin<T>::CH / 2 : TileWin<T>::CH; }

template <class T, int NB>
hipError_t interp2d_tile_nb(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    const PrecData<T>& d = prec<T>(P);
    const TileGeo<T> g = make_tile_geo<T>(P);
    const int nt = g.ntx * g.ntx;
    ProfScope _p(K_INTERP2D, s);
    hipLaunchKernelGGL((interp_tile_kernel<T, TileWin<T>::W, TileWin<T>::DEG, NB>), dim3(nt), dim3(256), 0, s, g,
                       d.grid, d.sr, d.sc, x, y, flags);
    return hipGetLastError();
}

template <class T, int NB>
hipError_t adjoint2d_tile_nb(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s) {
    const PrecData<T>& d = prec<T>(P);
    const TileGeo<T> g = make_tile_geo<T>(P);
    constexpr int W = TileWin<T>::W, DEG = TileWin<T>::DEG, CH = tile_chunk<T, NB>();
    constexpr int PW = TILE_TS + W - 1;
    const int nt = g.ntx * g.ntx;
    const int nch = 2 * P.nb;
    cx<T>* partI = d.part;
    cx<T>* partR = partI + (size_t)nt * PW * PW;
    cx<T>* partC = partR + (size_t)nt * nch * PW;
    cx<T>* partX = partC + (size_t)nt * nch * PW;
    {
        ProfScope _p(K_SPREAD2D, s);
        hipLaunchKernelGGL((adjoint_tile_kernel<T, W, DEG, NB, CH>), dim3(nt), dim3(384), 0, s, g, u, flags, partI,
                           partR, partC, partX);
        GS_HIP_TRY(hipGetLastError());
    }
    {
        ProfScope _p(K_MERGE, s);
        hipLaunchKernelGGL((merge_grid_kernel<T, W>), dim3((g.ng * g.ng + 255) / 256), dim3(256), 0, s, g, partI,
                           d.grid);
        GS_HIP_TRY(hipGetLastError());
        if (NB > 0) {
            hipLaunchKernelGGL((merge_sides_kernel<T, W>), dim3((2 * nch * g.ng + 255) / 256), dim3(256), 0, s, g,
                               partR, partC, d.sr, d.sc);
            GS_HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL((merge_corners_kernel<T>), dim3(nch * nch), dim3(256), 0, s, g, partX, nt, x);
            GS_HIP_TRY(hipGetLastError());
        }
    }
    return hipSuccess;
}

template <class T>
hipError_t interp2d_tile(const Plan& P, const cx<T>* x, cx<T>* y, int flags, hipStream_t s) {
    switch (P.nb) {
        case 0: return interp2d_tile_nb<T, 0>(P, x, y, flags, s);
        case 2: return interp2d_tile_nb<T, 2>(P, x, y, flags, s);
        case 3: return interp2d_tile_nb<T, 3>(P, x, y, flags, s);
        case 4: return interp2d_tile_nb<T, 4>(P, x, y, flags, s);
        case 5: return interp2d_tile_nb<T, 5>(P, x, y, flags, s);
        case 6: return interp2d_tile_nb<T, 6>(P, x, y, flags, s);
        case 7: return interp2d_tile_nb<T, 7>(P, x, y, flags, s);
        case 8: return interp2d_tile_nb<T, 8>(P, x, y, flags, s);
    }
    return hipErrorInvalidValue;
}

template <class T>
hipError_t adjoint2d_tile(const Plan& P, const cx<T>* u, cx<T>* x, int flags, hipStream_t s) {
    switch (P.nb) {
        case 0: return adjoint2d_tile_nb<T, 0>(P, u, x, flags, s);
        case 2: return adjoint2d_tile_nb<T, 2>(P, u, x, flags, s);
        case 3: return adjoint2d_tile_nb<T, 3>(P, u, x, flags, s);
        case 4: return adjoint2d_tile_nb<T, 4>(P, u, x, flags, s);
        case 5: return adjoint2d_tile_nb<T, 5>(P, u, x, flags, s);
        case 6: return adjoint2d_tile_nb<T, 6>(P, u, x, flags, s);
        case 7: return adjoint2d_tile_nb<T, 7>(P, u, x, flags, s);
        case 8: return adjoint2d_tile_nb<T, 8>(P, u, x, flags, s);
    }
    return hipErrorInvalidValue;
}

template hipError_t interp2d_tile<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t);
template hipError_t interp2d_tile<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t);
template hipError_t adjoint2d_tile<float>(const Plan&, const cx<float>*, cx<float>*, int, hipStream_t);
template hipError_t adjoint2d_tile<double>(const Plan&, const cx<double>*, cx<double>*, int, hipStream_t);

// partial-buffer elements needed by the 2D adjoint
size_t adjoint2d_part_elems(int ng, int ts, int nb, int w) {
    const size_t nt = (size_t)(ng / ts) * (ng / ts);
    const size_t pw = ts + w - 1;
    return nt * (pw * pw + 2 * (2 * nb) * pw + (2 * nb) * (2 * nb)) + 64;
}

}  // namespace gs
