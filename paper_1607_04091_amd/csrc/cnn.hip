// Learned CGLS warm start (this library's form; the paper starts CGLS from
// zero).  A small residual CNN maps the adjoint image A^H b = T^H W y of a 2D
// problem (two real channels: re, im) to an estimate of the least-squares
// solution, which gs_solve then takes as x0.
//
// Network: x = s * input (s a fixed positive scale, set by the caller);
// conv3x3 2->32, ReLU; 4 x (conv3x3 32->32, ReLU); conv3x3 32->2;
// output = x + last conv.  Convolutions are cross-correlations with zero
// padding 1 and no biases; weights w[ky][kx][ci][co] (tap t = 3 ky + kx).
// Loss: sum ||out - target||^2 / sum ||target||^2 over the batch.  Adam
// (Kingma and Ba, Algorithm 1) on FP32 master weights.
//
// Precision: activations and hidden-layer gradients are stored as bfloat16
// (round to nearest even from FP32), products use bf16 copies of the master
// weights, every sum accumulates in FP32.  The 32->32 layers (97% of the
// flops) run on MFMA (v_mfma_f32_16x16x16_bf16): forward and backward-data
// are one kernel (backward-data is a forward convolution with the taps
// mirrored and the channel roles swapped, done by the weight packing), the
// weight gradient is a second MFMA kernel whose contraction runs over
// pixels.  The thin first and last layers (2 channels on one side) are plain
// FP32 ALU kernels.  All reductions have a fixed order: results are bitwise
// reproducible.
//
// Layout: images are channels-last; an activation pixel is 32 bf16 = 64 B.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "prof.hpp"

namespace gs {
namespace cnn {

constexpr int CH = 32;                        // hidden channels
constexpr int NL = 6;                         // convolution layers
constexpr int TAPS = 9;
constexpr int P1 = TAPS * 2 * CH;             // first layer weights (576)
constexpr int PH = TAPS * CH * CH;            // hidden layer weights (9216)
constexpr int P6 = TAPS * CH * 2;             // last layer weights (576)
constexpr int NPARAM = P1 + 4 * PH + P6;      // 38016
constexpr int PACK = 18 * 2 * 64;             // MFMA fragments (uint2) per hidden layer
__host__ __device__ constexpr int poff(int l) { return l == 0 ? 0 : P1 + (l - 1) * PH; }

constexpr int TS = 16;                        // output tile side of the MFMA kernels
constexpr int HALO = TS + 2;
constexpr int PSTR = 36;                      // LDS pixel stride, halfwords (72 B: conflict-free 8 B reads)
constexpr int DW_WG = 512;                    // weight-gradient workgroups (partials)
constexpr int THIN_WG = 1024;                 // thin-gradient workgroups (one partial each)
constexpr int THIN_SEG = 64;                  // pixels per row segment in the thin gradient kernel
constexpr int LOSS_B = 256;
constexpr int DSTR = 260;                     // transposed delta tile: channel stride, halfwords
constexpr int ASTR = 292;                     // transposed activation tile (18 rows): channel stride

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2bf(float f) {      // round to nearest even (finite f)
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bflo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bfhi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ uint32_t pack2(float a, float b) { return f2bf(a) | (f2bf(b) << 16); }
__device__ __forceinline__ v4s as_v4s(uint2 u) {
    v4s r;
    r[0] = (short)(u.x & 0xFFFF);
    r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xFFFF);
    r[3] = (short)(u.y >> 16);
    return r;
}
__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const uint16_t* p, int64_t i) { return __uint_as_float((uint32_t)p[i] << 16); }

// ------------------------------------------------------------------ first layer (2 -> 32), ALU
// x = scale * input (FP32); a1 = bf16(relu(conv(x, w1))); keeps x in x0 (residual, weight gradient)
template <class TI>
__global__ void __launch_bounds__(256) first_kernel(const TI* __restrict__ in, float scale, float* __restrict__ x0,
                                                    uint16_t* __restrict__ a1, const float* __restrict__ wq, int B,
                                                    int H, int W) {
    // the workgroup's 256 x 64-byte output rows go through LDS so that each
    // store instruction writes 1 KB of consecutive bytes
    __shared__ uint4 so[256 * 5];   // row stride 5 x 16 B
    const int64_t n = (int64_t)B * H * W;
    const int64_t pix0 = (int64_t)blockIdx.x * 256;
    const int64_t pix = pix0 + threadIdx.x;
    if (pix < n) {
        const int x = (int)(pix % W);
        const int y = (int)((pix / W) % H);
        const int64_t b = pix / ((int64_t)W * H);
        float acc[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = 0.f;
        for (int ky = 0; ky < 3; ++ky) {
            const int yy = y + ky - 1;
            if (yy < 0 || yy >= H) continue;
            for (int kx = 0; kx < 3; ++kx) {
                const int xx = x + kx - 1;
                if (xx < 0 || xx >= W) continue;
                const int64_t q = (b * H + yy) * W + xx;
                const float v0 = (float)in[2 * q] * scale, v1 = (float)in[2 * q + 1] * scale;
                const float* w = wq + (ky * 3 + kx) * 2 * CH;   // wave-uniform: scalar loads
#pragma unroll
                for (int c = 0; c < CH; ++c) acc[c] = fmaf(v1, w[CH + c], fmaf(v0, w[c], acc[c]));
            }
        }
        x0[2 * pix] = (float)in[2 * pix] * scale;
        x0[2 * pix + 1] = (float)in[2 * pix + 1] * scale;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float* a = acc + 8 * q;
            so[threadIdx.x * 5 + q] =
                make_uint4(pack2(fmaxf(a[0], 0.f), fmaxf(a[1], 0.f)), pack2(fmaxf(a[2], 0.f), fmaxf(a[3], 0.f)),
                           pack2(fmaxf(a[4], 0.f), fmaxf(a[5], 0.f)), pack2(fmaxf(a[6], 0.f), fmaxf(a[7], 0.f)));
        }
    }
    __syncthreads();
    uint4* o = reinterpret_cast<uint4*>(a1 + pix0 * CH);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = i * 256 + threadIdx.x, r = c >> 2;
        if (pix0 + r < n) o[c] = so[r * 5 + (c & 3)];
    }
}

// ------------------------------------------------------------------ hidden 32 -> 32 convolution, MFMA
// A workgroup takes 16 x 16 output tiles of one image in turn (tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...); each 18 x 18 x 32 input tile (with
// halo, zero outside) is staged in LDS, and the next tile's loads are issued
// before the current tile is computed.  As a GEMM per tap t and
// input-channel half h: D[co][pixel] += W_t[co][ci] X[ci][pixel]; A operands
// (weights) come pre-packed per lane and stay in registers (36 fragments), B
// operands (4 channels of one pixel, 8 bytes) are read from LDS.  Wave w owns
// tile rows 4w..4w+3, i.e. 4 x 2 accumulators of 16 x 16.
// EPI 0: ReLU (forward); EPI 1: multiply by [mask > 0] (backward data).
template <int EPI>
__global__ void __launch_bounds__(256) conv32_kernel(const uint16_t* __restrict__ in, const uint2* __restrict__ wpack,
                                                     uint16_t* __restrict__ out, const uint16_t* __restrict__ mask,
                                                     int B, int H, int W, int tiles_x, int tiles_y) {
    __shared__ __align__(16) uint16_t tile[HALO * HALO * PSTR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the weight fragments are loaded once per workgroup; the workgroup then
    // walks tiles blockIdx.x, blockIdx.x + gridDim.x, ...
    v4s wf[18][2];
#pragma unroll
    for (int s = 0; s < 18; ++s)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) wf[s][mb] = as_v4s(wpack[(s * 2 + mb) * 64 + lane]);
    const int col = lane & 15, kq = lane >> 4;
    const int ntiles = tiles_x * tiles_y * B;
    constexpr int NLD = (HALO * HALO * 4 + 255) / 256;   // 16-byte loads per thread and tile
    uint4 nx[NLD];
    // loads of tile t's input (with halo) into registers; stored to LDS later,
    // so that they are in flight while the previous tile is computed
    auto fetch = [&](int t) {
        const int x0 = (t % tiles_x) * TS, y0 = (t / tiles_x % tiles_y) * TS;
        const int64_t b = t / tiles_x / tiles_y;
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int pl = c >> 2, part = c & 3;
            const int py = pl / HALO, px = pl - py * HALO;
            const int gy = y0 + py - 1, gx = x0 + px - 1;
            nx[i] = make_uint4(0, 0, 0, 0);
            if (c < HALO * HALO * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W)
                nx[i] = *reinterpret_cast<const uint4*>(in + ((b * H + gy) * W + gx) * CH + part * 8);
        }
    };
    if ((int)blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int x0 = (t % tiles_x) * TS, y0 = (t / tiles_x % tiles_y) * TS;
        const int64_t b = t / tiles_x / tiles_y;
        __syncthreads();   // the previous tile's reads of the LDS tile are done
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int c = threadIdx.x + 256 * i;
            if (c < HALO * HALO * 4) {
                uint2* d = reinterpret_cast<uint2*>(tile + (c >> 2) * PSTR + (c & 3) * 8);
                d[0] = make_uint2(nx[i].x, nx[i].y);
                d[1] = make_uint2(nx[i].z, nx[i].w);
            }
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);

        v4f acc[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) acc[r][mb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 18; ++s) {
            const int tap = s >> 1, h = s & 1, ky = tap / 3, kx = tap % 3;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wave * 4 + r;
                const uint2 u =
                    *reinterpret_cast<const uint2*>(tile + ((row + ky) * HALO + col + kx) * PSTR + h * 16 + kq * 4);
                const v4s bv = as_v4s(u);
                acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wf[s][0], bv, acc[r][0], 0, 0, 0);
                acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wf[s][1], bv, acc[r][1], 0, 0, 0);
            }
        }
        // lane holds D[co = 16 mb + 4 kq + j][pixel = col]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gy = y0 + wave * 4 + r, gx = x0 + col;
            if (gy >= H || gx >= W) continue;
            const int64_t pix = (b * H + gy) * W + gx;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int co = mb * 16 + kq * 4;
                float v0 = acc[r][mb][0], v1 = acc[r][mb][1], v2 = acc[r][mb][2], v3 = acc[r][mb][3];
                if (EPI == 0) {
                    v0 = fmaxf(v0, 0.f);
                    v1 = fmaxf(v1, 0.f);
                    v2 = fmaxf(v2, 0.f);
                    v3 = fmaxf(v3, 0.f);
                } else {
                    const uint2 m = *reinterpret_cast<const uint2*>(mask + pix * CH + co);
                    v0 = bflo(m.x) > 0.f ? v0 : 0.f;
                    v1 = bfhi(m.x) > 0.f ? v1 : 0.f;
                    v2 = bflo(m.y) > 0.f ? v2 : 0.f;
                    v3 = bfhi(m.y) > 0.f ? v3 : 0.f;
                }
                *reinterpret_cast<uint2*>(out + pix * CH + co) = make_uint2(pack2(v0, v1), pack2(v2, v3));
            }
        }
    }
}

// ------------------------------------------------------------------ last layer (32 -> 2), ALU
// out = x0 + conv(a5, w6) in FP32; written to the FP32 buffer and/or the caller's output
template <class TO>
__global__ void __launch_bounds__(256) last_kernel(const uint16_t* __restrict__ a5, const float* __restrict__ x0,
                                                   const float* __restrict__ wq, float* __restrict__ outf,
                                                   TO* __restrict__ out, int B, int H, int W, int tiles_x,
                                                   int tiles_y) {
    // one 16 x 16 pixel tile per workgroup; its 18 x 18 x 32 input (with halo,
    // zero outside) is staged in LDS with coalesced loads
    __shared__ __align__(16) uint16_t tile[HALO * HALO * PSTR];
    int t = blockIdx.x;
    const int tx0 = (t % tiles_x) * TS;
    t /= tiles_x;
    const int ty0 = (t % tiles_y) * TS;
    const int64_t b = t / tiles_y;
    for (int c = threadIdx.x; c < HALO * HALO * 4; c += 256) {
        const int pl = c >> 2, part = c & 3;
        const int py = pl / HALO, px = pl - py * HALO;
        const int gy = ty0 + py - 1, gx = tx0 + px - 1;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const uint4*>(a5 + ((b * H + gy) * W + gx) * CH + part * 8);
        uint2* d = reinterpret_cast<uint2*>(tile + pl * PSTR + part * 8);
        d[0] = make_uint2(v.x, v.y);
        d[1] = make_uint2(v.z, v.w);
    }
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x >= W || y >= H) return;
    float acc0 = 0.f, acc1 = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int yy = y + ky - 1;
        if (yy < 0 || yy >= H) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int xx = x + kx - 1;
            if (xx < 0 || xx >= W) continue;
            const uint16_t* p = tile + ((ly + ky) * HALO + lx + kx) * PSTR;
            const float* w = wq + (ky * 3 + kx) * CH * 2;   // wave-uniform: scalar loads
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint2 v = *reinterpret_cast<const uint2*>(p + 4 * q);
                const uint32_t wd[2] = {v.x, v.y};
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int ci = 4 * q + 2 * e;
                    const float lo = bflo(wd[e]), hi = bfhi(wd[e]);
                    acc0 = fmaf(lo, w[2 * ci], acc0);
                    acc1 = fmaf(lo, w[2 * ci + 1], acc1);
                    acc0 = fmaf(hi, w[2 * ci + 2], acc0);
                    acc1 = fmaf(hi, w[2 * ci + 3], acc1);
                }
            }
        }
    }
    const int64_t pix = (b * H + y) * W + x;
    const float o0 = x0[2 * pix] + acc0, o1 = x0[2 * pix + 1] + acc1;
    if (outf) {
        outf[2 * pix] = o0;
        outf[2 * pix + 1] = o1;
    }
    if (out) {
        out[2 * pix] = (TO)o0;
        out[2 * pix + 1] = (TO)o1;
    }
}

// ------------------------------------------------------------------ loss and its gradient
template <class TT>
__global__ void __launch_bounds__(256) loss_partial_kernel(const float* __restrict__ out, const TT* __restrict__ tgt,
                                                           int64_t n, double* __restrict__ part) {
    __shared__ double s0[256], s1[256];
    double d2 = 0, t2 = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)LOSS_B * 256) {
        const double t = (double)tgt[i];
        const double d = (double)out[i] - t;
        d2 += d * d;
        t2 += t * t;
    }
    s0[threadIdx.x] = d2;
    s1[threadIdx.x] = t2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0[0];
        part[LOSS_B + blockIdx.x] = s1[0];
    }
}

// scal[0] = sum d^2, scal[1] = sum t^2, scal[2] = loss
__global__ void __launch_bounds__(256) loss_final_kernel(const double* __restrict__ part, double* __restrict__ scal) {
    __shared__ double s0[256], s1[256];
    s0[threadIdx.x] = part[threadIdx.x];
    s1[threadIdx.x] = part[LOSS_B + threadIdx.x];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[0] = s0[0];
        scal[1] = s1[0];
        scal[2] = s1[0] > 0 ? s0[0] / s1[0] : 0.0;
    }
}

// d6 = 2 (out - target) / sum ||target||^2
template <class TT>
__global__ void __launch_bounds__(256) delta_out_kernel(const float* __restrict__ out, const TT* __restrict__ tgt,
                                                        const double* __restrict__ scal, float* __restrict__ d6,
                                                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double S = scal[1];
    d6[i] = S > 0 ? (float)(2.0 * ((double)out[i] - (double)tgt[i]) / S) : 0.f;
}

// ------------------------------------------------------------------ last layer backward data, ALU
// d5[q][ci] = bf16( [a5[q][ci] > 0] * sum_t sum_co d6[q - t][co] w6[t][ci][co] )
__global__ void __launch_bounds__(256) last_bwd_kernel(const float* __restrict__ d6, const float* __restrict__ wq,
                                                       const uint16_t* __restrict__ a5, uint16_t* __restrict__ d5,
                                                       int B, int H, int W) {
    const int64_t n = (int64_t)B * H * W;
    const int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= n) return;
    const int x = (int)(pix % W);
    const int y = (int)((pix / W) % H);
    const int64_t b = pix / ((int64_t)W * H);
    float g[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) g[c] = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int yy = y - (ky - 1);
        if (yy < 0 || yy >= H) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int xx = x - (kx - 1);
            if (xx < 0 || xx >= W) continue;
            const int64_t q = (b * H + yy) * W + xx;
            const float e0 = d6[2 * q], e1 = d6[2 * q + 1];
            const float* w = wq + (ky * 3 + kx) * CH * 2;   // wave-uniform: scalar loads
#pragma unroll
            for (int c = 0; c < CH; ++c) g[c] = fmaf(e1, w[2 * c + 1], fmaf(e0, w[2 * c], g[c]));
        }
    }
    const uint4* mp = reinterpret_cast<const uint4*>(a5 + pix * CH);
    uint4* o = reinterpret_cast<uint4*>(d5 + pix * CH);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 m = mp[q];
        const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
        uint32_t r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 8 * q + 2 * e;
            r[e] = pack2(bflo(mw[e]) > 0.f ? g[c] : 0.f, bfhi(mw[e]) > 0.f ? g[c + 1] : 0.f);
        }
        o[q] = make_uint4(r[0], r[1], r[2], r[3]);
    }
}

// ------------------------------------------------------------------ hidden weight gradient, MFMA
// dW[t][ci][co] = sum over pixels p of a[p + t][ci] d[p][co].  Per tap, a GEMM
// D[co][ci] += dT[co][p] a_t[p][ci] whose contraction runs over the 16 pixels of
// a tile row.  Tiles are staged transposed (channel-major, pixels contiguous)
// so that a lane's 4 consecutive pixels are one 8-byte read; the activation
// tile is kept in three copies shifted by kx = 0, 1, 2 so every read is
// aligned.  Wave w owns (co block w >> 1, ci block w & 1) for all 9 taps.
// Workgroups loop over tiles, issuing the next tile's global loads before
// computing the current one; each writes one FP32 partial of all 9216
// gradients, summed afterwards in a fixed order.
__global__ void __launch_bounds__(256) dw32_kernel(const uint16_t* __restrict__ act, const uint16_t* __restrict__ dlt,
                                                   float* __restrict__ part, int B, int H, int W, int tiles_x,
                                                   int tiles_y) {
    __shared__ __align__(16) uint16_t Dt[CH * DSTR];
    __shared__ __align__(16) uint16_t As[3 * CH * ASTR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mb = wave >> 1, nb = wave & 1;
    const int c16 = lane & 15, kq = lane >> 4;
    v4f acc[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t ntiles = (int64_t)tiles_x * tiles_y * B;
    constexpr int NDL = TS * TS * 4 / 256, NAL = (HALO * HALO * 4 + 255) / 256;   // 16-byte loads per thread
    static_assert(TS * TS * 4 % 256 == 0, "whole d-tile loads");
    uint4 nd[NDL], na[NAL];
    // loads of tile tl's d values and activations (with halo) into registers;
    // stored to LDS later, so that they are in flight while the previous tile
    // is computed
    auto fetch = [&](int64_t tl) {
        const int x0 = (int)(tl % tiles_x) * TS, y0 = (int)(tl / tiles_x % tiles_y) * TS;
        const int64_t b = tl / tiles_x / tiles_y;
#pragma unroll
        for (int i = 0; i < NDL; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int pl = c >> 2, part8 = (c & 3) * 8;
            const int gy = y0 + (pl >> 4), gx = x0 + (pl & 15);
            nd[i] = make_uint4(0, 0, 0, 0);
            if (gy < H && gx < W) nd[i] = *reinterpret_cast<const uint4*>(dlt + ((b * H + gy) * W + gx) * CH + part8);
        }
#pragma unroll
        for (int i = 0; i < NAL; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int pl = c >> 2, part8 = (c & 3) * 8;
            const int py = pl / HALO, px = pl - py * HALO;
            const int gy = y0 + py - 1, gx = x0 + px - 1;
            na[i] = make_uint4(0, 0, 0, 0);
            if (c < HALO * HALO * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W)
                na[i] = *reinterpret_cast<const uint4*>(act + ((b * H + gy) * W + gx) * CH + part8);
        }
    };
    if ((int64_t)blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        __syncthreads();   // the previous tile's reads of Dt and As are done
#pragma unroll
        for (int i = 0; i < NDL; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int pl = c >> 2, part8 = (c & 3) * 8;
            const int ry = pl >> 4, rx = pl & 15;
            const uint32_t w4[4] = {nd[i].x, nd[i].y, nd[i].z, nd[i].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Dt[(part8 + 2 * e) * DSTR + ry * TS + rx] = (uint16_t)(w4[e] & 0xFFFF);
                Dt[(part8 + 2 * e + 1) * DSTR + ry * TS + rx] = (uint16_t)(w4[e] >> 16);
            }
        }
#pragma unroll
        for (int i = 0; i < NAL; ++i) {
            const int c = threadIdx.x + 256 * i;
            if (c >= HALO * HALO * 4) continue;
            const int pl = c >> 2, part8 = (c & 3) * 8;
            const int py = pl / HALO, px = pl - py * HALO;
            const uint32_t w4[4] = {na[i].x, na[i].y, na[i].z, na[i].w};
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int xp = px - s;
                if (xp < 0 || xp >= TS) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    As[(s * CH + part8 + 2 * e) * ASTR + py * TS + xp] = (uint16_t)(w4[e] & 0xFFFF);
                    As[(s * CH + part8 + 2 * e + 1) * ASTR + py * TS + xp] = (uint16_t)(w4[e] >> 16);
                }
            }
        }
        __syncthreads();
        if (tl + gridDim.x < ntiles) fetch(tl + gridDim.x);
        for (int rho = 0; rho < TS; ++rho) {
            const v4s av = as_v4s(*reinterpret_cast<const uint2*>(Dt + (16 * mb + c16) * DSTR + rho * TS + 4 * kq));
#pragma unroll
            for (int tap = 0; tap < TAPS; ++tap) {
                const int ky = tap / 3, kx = tap % 3;
                const v4s bv = as_v4s(*reinterpret_cast<const uint2*>(
                    As + (kx * CH + 16 * nb + c16) * ASTR + (rho + ky) * TS + 4 * kq));
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[tap], 0, 0, 0);
            }
        }
    }
    // lane holds D[co = 16 mb + 4 kq + j][ci = 16 nb + c16]
    float* P = part + (int64_t)blockIdx.x * PH;
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap)
#pragma unroll
        for (int j = 0; j < 4; ++j) P[(tap * CH + 16 * nb + c16) * CH + 16 * mb + 4 * kq + j] = acc[tap][j];
}

// ------------------------------------------------------------------ thin-layer weight gradients, ALU
// dW[t][cu][cv] = sum_p U[p + t][cu] V[p][cv] with CU * CV = 64.  A workgroup
// takes row segments of THIN_SEG pixels in turn.  It stages the segment's three
// input rows of U (one extra pixel either side, zero outside the image) and its
// V values in LDS with 16- or 8-byte loads, then wave w sums pixels
// THIN_CH w .. THIN_CH w + THIN_CH - 1 of the segment: lane (cu, cv) owns the 9
// taps of one (cu, cv) pair and reads the 3 x (THIN_CH + 2) values of U and the
// THIN_CH values of V it needs into registers.  The four waves add their sums in
// LDS in a fixed order; one partial per workgroup.
constexpr int THIN_CH = THIN_SEG / 4;
template <int NB> struct VecOf;
template <> struct VecOf<16> {
    using type = uint4;
    __device__ static type zero() { return make_uint4(0, 0, 0, 0); }
};
template <> struct VecOf<8> {
    using type = uint2;
    __device__ static type zero() { return make_uint2(0, 0); }
};

template <int CU, int CV, class UT, class VT>
__global__ void __launch_bounds__(256) dw_thin_kernel(const UT* __restrict__ U, const VT* __restrict__ V,
                                                      float* __restrict__ part, int B, int H, int W, int segs_x) {
    static_assert(CU * CV == 64, "one (cu, cv) pair per lane");
    constexpr int UPX = CU * (int)sizeof(UT), VPX = CV * (int)sizeof(VT);     // bytes per pixel
    constexpr int UVB = UPX >= 16 ? 16 : UPX, VVB = VPX >= 16 ? 16 : VPX;       // bytes per load
    static_assert(UPX % UVB == 0 && VPX % VVB == 0 && (UVB == 16 || UVB == 8) && (VVB == 16 || VVB == 8),
                  "pixel rows load as whole 8- or 16-byte vectors");
    using UVec = typename VecOf<UVB>::type;
    using VVec = typename VecOf<VVB>::type;
    constexpr int SEGU = THIN_SEG + 2;
    __shared__ __align__(16) unsigned char su[3 * SEGU * UPX];
    __shared__ __align__(16) unsigned char sv[THIN_SEG * VPX];
    __shared__ float red[4][TAPS * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cu = lane / CV, cv = lane % CV;
    const UT* lu = reinterpret_cast<const UT*>(su);
    const VT* lv = reinterpret_cast<const VT*>(sv);
    const int64_t nseg = (int64_t)B * H * segs_x;
    float acc[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) acc[t] = 0.f;
    for (int64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int sx = (int)(sg % segs_x);
        const int y = (int)((sg / segs_x) % H);
        const int64_t b = sg / ((int64_t)segs_x * H);
        const int x0 = sx * THIN_SEG;
        __syncthreads();   // the previous segment's reads of su and sv are done
        constexpr int UPV = UPX / UVB, VPV = VPX / VVB;   // loads per pixel
        for (int c = threadIdx.x; c < 3 * SEGU * UPV; c += 256) {
            const int r = c / (SEGU * UPV), px = (c / UPV) % SEGU, k = c % UPV;
            const int yy = y + r - 1, x = x0 - 1 + px;
            UVec v = VecOf<UVB>::zero();
            if (yy >= 0 && yy < H && x >= 0 && x < W)
                v = reinterpret_cast<const UVec*>(U + ((b * H + yy) * W + x) * CU)[k];
            reinterpret_cast<UVec*>(su)[c] = v;
        }
        for (int c = threadIdx.x; c < THIN_SEG * VPV; c += 256) {
            const int px = c / VPV, k = c % VPV;
            const int x = x0 + px;
            VVec v = VecOf<VVB>::zero();
            if (x < W) v = reinterpret_cast<const VVec*>(V + ((b * H + y) * W + x) * CV)[k];
            reinterpret_cast<VVec*>(sv)[c] = v;
        }
        __syncthreads();
        const int k0 = wave * THIN_CH;
        float u[3][THIN_CH + 2], v[THIN_CH];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < THIN_CH + 2; ++k) u[r][k] = ldv(lu, (r * SEGU + k0 + k) * CU + cu);
#pragma unroll
        for (int k = 0; k < THIN_CH; ++k) v[k] = ldv(lv, (k0 + k) * CV + cv);
#pragma unroll
        for (int k = 0; k < THIN_CH; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) acc[r * 3 + kx] = fmaf(u[r][k + kx], v[k], acc[r * 3 + kx]);
    }
#pragma unroll
    for (int t = 0; t < TAPS; ++t) red[wave][t * 64 + lane] = acc[t];
    __syncthreads();
    for (int i = threadIdx.x; i < TAPS * 64; i += 256) {
        const int t = i >> 6, l = i & 63;
        const float sum = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
        part[(int64_t)blockIdx.x * (TAPS * 64) + (t * CU + l / CV) * CV + l % CV] = sum;
    }
}

// Sum of nparts partials of `count` values in a fixed order, in two stages:
// stage 1 sums the partials of each of RED_G groups (block (x, g) covers 256
// consecutive values of group g), stage 2 sums the RED_G group sums.
constexpr int RED_G = 32;
__global__ void __launch_bounds__(256) dw_reduce1_kernel(const float* __restrict__ part, int nparts, int count,
                                                         float* __restrict__ tmp) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int g = blockIdx.y;
    if (i >= count) return;
    const int per = (nparts + RED_G - 1) / RED_G;
    const int p0 = g * per, p1 = min(nparts, p0 + per);
    float s = 0.f;
    for (int p = p0; p < p1; ++p) s += part[(int64_t)p * count + i];
    tmp[(int64_t)g * count + i] = s;
}

__global__ void __launch_bounds__(256) dw_reduce2_kernel(const float* __restrict__ tmp, int count,
                                                         float* __restrict__ grad) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
#pragma unroll 8
    for (int g = 0; g < RED_G; ++g) s += tmp[(int64_t)g * count + i];
    grad[i] = s;
}

// ------------------------------------------------------------------ optimizer and weight packing
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, int n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// MFMA A fragments of the hidden layers (lane l of fragment (s, mb) holds
// W[t][16h + 4(l>>4) + j][16mb + (l&15)], j = 0..3, t = s>>1, h = s&1), for the
// forward weights and for the backward-data weights W'[t][c][k] = W[8-t][k][c];
// plus bf16-rounded FP32 copies of the thin layers
__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ w, uint2* __restrict__ fwd,
                                                   uint2* __restrict__ bwd, float* __restrict__ wq1,
                                                   float* __restrict__ wq6) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 4 * PACK) {
        const int l = i / PACK, r = i % PACK;
        const int lane = r & 63, sm = r >> 6, s = sm >> 1, mb = sm & 1, tap = s >> 1, h = s & 1;
        const float* Wl = w + poff(l + 1);
        float f[4], g[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ci = 16 * h + 4 * (lane >> 4) + j, co = 16 * mb + (lane & 15);
            f[j] = Wl[(tap * CH + ci) * CH + co];
            g[j] = Wl[((8 - tap) * CH + co) * CH + ci];
        }
        fwd[i] = make_uint2(pack2(f[0], f[1]), pack2(f[2], f[3]));
        bwd[i] = make_uint2(pack2(g[0], g[1]), pack2(g[2], g[3]));
    }
    if (i < P1) wq1[i] = __uint_as_float(f2bf(w[i]) << 16);
    if (i < P6) wq6[i] = __uint_as_float(f2bf(w[poff(5) + i]) << 16);
}

struct Net {
    int H = 0, W = 0, maxB = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint2 *fwd = nullptr, *bwd = nullptr;
    float *wq1 = nullptr, *wq6 = nullptr;
    uint16_t* act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    uint16_t* dl[2] = {nullptr, nullptr};
    float *x0 = nullptr, *outf = nullptr, *d6 = nullptr, *part = nullptr, *red = nullptr;
    double *lpart = nullptr, *lscal = nullptr, *host = nullptr;
    int step = 0;
    float in_scale = 1.f;      // fixed input scale (not trained)
    int train_batch = 0;       // batch of the last training forward (0: none)
    int conv_wg = 512;         // workgroups of a convolution launch: two per compute unit
    std::vector<void*> allocs;
};

inline int64_t pix_count(const Net& n, int batch) { return (int64_t)batch * n.H * n.W; }
inline int nblk(int64_t n, int t = 256) { return (int)std::max<int64_t>(1, (n + t - 1) / t); }
// workgroups of the convolution kernels (each walks tiles, reusing its weight
// fragments and prefetching the next tile): one resident round, two per CU
inline int conv_grid(const Net& n, int tiles) { return std::min(tiles, n.conv_wg); }

}  // namespace cnn
}  // namespace gs

struct gs_cnn {
    gs::cnn::Net net;
};

using namespace gs;
using namespace gs::cnn;

static void cnn_free(gs_cnn_t* c) {
    if (!c) return;
    for (void* p : c->net.allocs) (void)hipFree(p);
    if (c->net.host) (void)hipHostFree(c->net.host);
    delete c;
}

extern "C" int gs_cnn_param_count(void) { return NPARAM; }

extern "C" int gs_cnn_create(gs_cnn_t** out, int height, int width, int max_batch) {
    if (!out) return GS_ERR_INVALID_ARG;
    *out = nullptr;
    if (height < 1 || width < 1 || height > 8192 || width > 8192 || max_batch < 1 || max_batch > 4096)
        return GS_ERR_INVALID_ARG;
    auto* c = new (std::nothrow) gs_cnn;
    if (!c) return GS_ERR_NOMEM;
    Net& n = c->net;
    n.H = height;
    n.W = width;
    n.maxB = max_batch;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            n.conv_wg = 2 * cus;
    }
    const int64_t np = (int64_t)max_batch * height * width;
    bool ok = true;
    auto alloc = [&](auto*& ptr, int64_t count) {
        void* p = nullptr;
        if (ok && hipMalloc(&p, (size_t)count * sizeof(*ptr)) == hipSuccess) {
            ptr = static_cast<std::remove_reference_t<decltype(ptr)>>(p);
            n.allocs.push_back(p);
        } else {
            ok = false;
        }
    };
    alloc(n.w, NPARAM);
    alloc(n.m, NPARAM);
    alloc(n.v, NPARAM);
    alloc(n.g, NPARAM);
    alloc(n.fwd, 4 * PACK);
    alloc(n.bwd, 4 * PACK);
    alloc(n.wq1, P1);
    alloc(n.wq6, P6);
    for (auto& a : n.act) alloc(a, np * CH);
    for (auto& d : n.dl) alloc(d, np * CH);
    alloc(n.x0, np * 2);
    alloc(n.outf, np * 2);
    alloc(n.d6, np * 2);
    alloc(n.part, (int64_t)std::max(DW_WG * PH, THIN_WG * 576));
    alloc(n.red, (int64_t)RED_G * PH);
    alloc(n.lpart, 2 * LOSS_B);
    alloc(n.lscal, 4);
    if (ok && hipHostMalloc((void**)&n.host, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) ok = false;
    if (!ok) {
        cnn_free(c);
        return GS_ERR_NOMEM;
    }
    for (float* p : {n.w, n.m, n.v, n.g})
        if (hipMemset(p, 0, NPARAM * sizeof(float)) != hipSuccess) ok = false;
    hipLaunchKernelGGL(pack_kernel, dim3(nblk(4 * PACK)), dim3(256), 0, nullptr, n.w, n.fwd, n.bwd, n.wq1, n.wq6);
    if (!ok || hipDeviceSynchronize() != hipSuccess) {
        cnn_free(c);
        return GS_ERR_HIP;
    }
    *out = c;
    return GS_OK;
}

extern "C" void gs_cnn_destroy(gs_cnn_t* c) { cnn_free(c); }

extern "C" int gs_cnn_set_input_scale(gs_cnn_t* c, float scale) {
    if (!c || !std::isfinite(scale) || !(scale > 0.f)) return GS_ERR_INVALID_ARG;
    c->net.in_scale = scale;
    c->net.train_batch = 0;
    return GS_OK;
}

extern "C" int gs_cnn_get_input_scale(const gs_cnn_t* c, float* scale) {
    if (!c || !scale) return GS_ERR_INVALID_ARG;
    *scale = c->net.in_scale;
    return GS_OK;
}

extern "C" int gs_cnn_set_weights(gs_cnn_t* c, const float* host) {
    if (!c || !host) return GS_ERR_INVALID_ARG;
    Net& n = c->net;
    for (int i = 0; i < NPARAM; ++i)
        if (!std::isfinite(host[i])) return GS_ERR_INVALID_ARG;
    if (hipMemcpy(n.w, host, NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return GS_ERR_HIP;
    if (hipMemset(n.m, 0, NPARAM * sizeof(float)) != hipSuccess) return GS_ERR_HIP;
    if (hipMemset(n.v, 0, NPARAM * sizeof(float)) != hipSuccess) return GS_ERR_HIP;
    n.step = 0;
    n.train_batch = 0;
    hipLaunchKernelGGL(pack_kernel, dim3(nblk(4 * PACK)), dim3(256), 0, nullptr, n.w, n.fwd, n.bwd, n.wq1, n.wq6);
    return hipDeviceSynchronize() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

static int copy_out(const float* dev, float* host) {
    if (!host) return GS_ERR_INVALID_ARG;
    return hipMemcpy(host, dev, NPARAM * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? GS_OK : GS_ERR_HIP;
}

extern "C" int gs_cnn_get_weights(const gs_cnn_t* c, float* host) { return c ? copy_out(c->net.w, host) : GS_ERR_INVALID_ARG; }
extern "C" int gs_cnn_get_grads(const gs_cnn_t* c, float* host) { return c ? copy_out(c->net.g, host) : GS_ERR_INVALID_ARG; }

extern "C" int gs_cnn_get_state(const gs_cnn_t* c, float* m, float* v, int* step) {
    if (!c || !step) return GS_ERR_INVALID_ARG;
    int rc = copy_out(c->net.m, m);
    if (rc == GS_OK) rc = copy_out(c->net.v, v);
    *step = c->net.step;
    return rc;
}

extern "C" int gs_cnn_set_state(gs_cnn_t* c, const float* m, const float* v, int step) {
    if (!c || !m || !v || step < 0) return GS_ERR_INVALID_ARG;
    Net& n = c->net;
    if (hipMemcpy(n.m, m, NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return GS_ERR_HIP;
    if (hipMemcpy(n.v, v, NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return GS_ERR_HIP;
    n.step = step;
    return GS_OK;
}

extern "C" int gs_cnn_forward(gs_cnn_t* c, const void* in, void* out, int batch, int flags, void* stream) {
    if (!c || !in || batch < 1 || batch > c->net.maxB) return GS_ERR_INVALID_ARG;
    if (flags & ~(GS_CNN_IN_F64 | GS_CNN_OUT_F64 | GS_CNN_TRAIN)) return GS_ERR_INVALID_ARG;
    if (!out && !(flags & GS_CNN_TRAIN)) return GS_ERR_INVALID_ARG;
    Net& n = c->net;
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = pix_count(n, batch);
    const int tx = (n.W + TS - 1) / TS, ty = (n.H + TS - 1) / TS;
    const int tiles = tx * ty * batch;
    {
    ProfScope _p(K_CNN_FIRST, st);
    if (flags & GS_CNN_IN_F64)
        hipLaunchKernelGGL((first_kernel<double>), dim3(nblk(np)), dim3(256), 0, st, (const double*)in, n.in_scale, n.x0,
                           n.act[0], n.wq1, batch, n.H, n.W);
    else
        hipLaunchKernelGGL((first_kernel<float>), dim3(nblk(np)), dim3(256), 0, st, (const float*)in, n.in_scale, n.x0,
                           n.act[0], n.wq1, batch, n.H, n.W);
    }
    for (int l = 0; l < 4; ++l) {
        ProfScope _p(K_CNN_CONV, st);
        hipLaunchKernelGGL((conv32_kernel<0>), dim3(conv_grid(n, tiles)), dim3(256), 0, st, n.act[l], n.fwd + l * PACK,
                           n.act[l + 1], (const uint16_t*)nullptr, batch, n.H, n.W, tx, ty);
    }
    float* outf = (flags & GS_CNN_TRAIN) ? n.outf : nullptr;
    ProfScope _p(K_CNN_LAST, st);
    if (flags & GS_CNN_OUT_F64)
        hipLaunchKernelGGL((last_kernel<double>), dim3(tiles), dim3(256), 0, st, n.act[4], n.x0, n.wq6, outf,
                           (double*)out, batch, n.H, n.W, tx, ty);
    else
        hipLaunchKernelGGL((last_kernel<float>), dim3(tiles), dim3(256), 0, st, n.act[4], n.x0, n.wq6, outf,
                           (float*)out, batch, n.H, n.W, tx, ty);
    if (hipGetLastError() != hipSuccess) return GS_ERR_HIP;
    n.train_batch = (flags & GS_CNN_TRAIN) ? batch : 0;
    return GS_OK;
}

extern "C" int gs_cnn_backward(gs_cnn_t* c, const void* target, int batch, int flags, double* loss, void* stream) {
    if (!c || !target || batch < 1) return GS_ERR_INVALID_ARG;
    if (flags & ~GS_CNN_TGT_F64) return GS_ERR_INVALID_ARG;
    Net& n = c->net;
    if (n.train_batch != batch) return GS_ERR_INVALID_ARG;   // needs the training forward of this batch
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = pix_count(n, batch);
    const int tx = (n.W + TS - 1) / TS, ty = (n.H + TS - 1) / TS;
    const int tiles = tx * ty * batch;
    const int dw_wg = std::min(DW_WG, tiles);
    const int segs_x = (n.W + THIN_SEG - 1) / THIN_SEG;
    const int thin_wg = (int)std::min<int64_t>(THIN_WG, (int64_t)batch * n.H * segs_x);
    auto reduce = [&](int nparts, int count, float* out) {
        hipLaunchKernelGGL(dw_reduce1_kernel, dim3(nblk(count), RED_G), dim3(256), 0, st, n.part, nparts, count,
                           n.red);
        hipLaunchKernelGGL(dw_reduce2_kernel, dim3(nblk(count)), dim3(256), 0, st, n.red, count, out);
    };
    // loss and d6
    {
    ProfScope _p(K_CNN_LOSS, st);
    if (flags & GS_CNN_TGT_F64) {
        hipLaunchKernelGGL((loss_partial_kernel<double>), dim3(LOSS_B), dim3(256), 0, st, n.outf,
                           (const double*)target, 2 * np, n.lpart);
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, n.lpart, n.lscal);
        hipLaunchKernelGGL((delta_out_kernel<double>), dim3(nblk(2 * np)), dim3(256), 0, st, n.outf,
                           (const double*)target, n.lscal, n.d6, 2 * np);
    } else {
        hipLaunchKernelGGL((loss_partial_kernel<float>), dim3(LOSS_B), dim3(256), 0, st, n.outf, (const float*)target,
                           2 * np, n.lpart);
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, n.lpart, n.lscal);
        hipLaunchKernelGGL((delta_out_kernel<float>), dim3(nblk(2 * np)), dim3(256), 0, st, n.outf,
                           (const float*)target, n.lscal, n.d6, 2 * np);
    }
    }
    // layer 6: weight gradient, then data gradient into d5
    {
        ProfScope _p(K_CNN_DW_THIN, st);
        hipLaunchKernelGGL((dw_thin_kernel<CH, 2, uint16_t, float>), dim3(thin_wg), dim3(256), 0, st, n.act[4],
                           n.d6, n.part, batch, n.H, n.W, segs_x);
        reduce(thin_wg, P6, n.g + poff(5));
    }
    {
        ProfScope _p(K_CNN_LAST_BWD, st);
        hipLaunchKernelGGL(last_bwd_kernel, dim3(nblk(np)), dim3(256), 0, st, n.d6, n.wq6, n.act[4], n.dl[0], batch,
                           n.H, n.W);
    }
    // hidden layers 5..2 (1-based): weight gradient, then masked data gradient
    int cur = 0;
    for (int l = 5; l >= 2; --l) {
        const uint16_t* a_prev = n.act[l - 2];
        {
            ProfScope _p(K_CNN_DW, st);
            hipLaunchKernelGGL(dw32_kernel, dim3(dw_wg), dim3(256), 0, st, a_prev, n.dl[cur], n.part, batch, n.H, n.W,
                               tx, ty);
            reduce(dw_wg, PH, n.g + poff(l - 1));
        }
        ProfScope _p(K_CNN_CONV_BWD, st);
        hipLaunchKernelGGL((conv32_kernel<1>), dim3(conv_grid(n, tiles)), dim3(256), 0, st, n.dl[cur], n.bwd + (l - 2) * PACK,
                           n.dl[cur ^ 1], a_prev, batch, n.H, n.W, tx, ty);
        cur ^= 1;
    }
    // layer 1: weight gradient from the FP32 input and d1
    {
        ProfScope _p(K_CNN_DW_THIN, st);
        hipLaunchKernelGGL((dw_thin_kernel<2, CH, float, uint16_t>), dim3(thin_wg), dim3(256), 0, st, n.x0,
                           n.dl[cur], n.part, batch, n.H, n.W, segs_x);
        reduce(thin_wg, P1, n.g + poff(0));
    }
    if (hipGetLastError() != hipSuccess) return GS_ERR_HIP;
    if (loss) {
        if (hipMemcpyAsync(n.host, n.lscal, 4 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return GS_ERR_HIP;
        *loss = n.host[2];
    }
    return GS_OK;
}

extern "C" int gs_cnn_step(gs_cnn_t* c, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!c || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return GS_ERR_INVALID_ARG;
    Net& n = c->net;
    hipStream_t st = (hipStream_t)stream;
    n.step += 1;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, n.step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, n.step));
    ProfScope _p(K_CNN_STEP, st);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(NPARAM)), dim3(256), 0, st, n.w, n.m, n.v, n.g, NPARAM, lr, beta1,
                       beta2, eps, bc1, bc2);
    hipLaunchKernelGGL(pack_kernel, dim3(nblk(4 * PACK)), dim3(256), 0, st, n.w, n.fwd, n.bwd, n.wq1, n.wq6);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}
