// Plan construction on the device (the paper's "init", Table 1; Sec. 6.3):
// fixed-point wrapped nodes and cell keys, a stable sort of the points by
// cell, the cell offsets, and the per-point basis tables -- the interior scale
// D = 2^{-J/2} phi-hat(eta) as the product of m0 over dyadic dilations (App. A)
// and the boundary transforms by the dilation recursion
// v1(zeta) = U v1(zeta/2) + V v2(zeta/2) started from v1(0) (App. A.1) -- for
// every point and dimension, written in sorted order in each precision the
// plan holds.  Only the frequencies and weights cross PCIe.
//
// The filters (taps, U, V, v1(0)) come from the host construction; the
// per-point arithmetic follows the host evaluation step for step in FP64, so
// the two agree to rounding (about 1e-15).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "host_math.hpp"

namespace gs {

namespace {

constexpr int PLAN_THREADS = 256;

// fixed-point wrapped node: round(frac(2^-J xi) 2^64), the same value the
// host computes in extended precision (2^-J xi, its fractional part and the
// scaling by 2^64 are exact in FP64; the rounding is to nearest, ties even)
__device__ inline uint64_t fixed_node(double xi, int J) {
    const double eta = ldexp(xi, -J);
    const double f = eta - floor(eta);
    return (uint64_t)rint(ldexp(f, 64));
}

__global__ void keys_kernel(const double* __restrict__ xi, int64_t M, int dim, int J, int G, int ts, int ng,
                            uint64_t* __restrict__ u, int32_t* __restrict__ key, int32_t* __restrict__ idx) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    int64_t cell[2] = {0, 0};
    for (int d = 0; d < dim; ++d) {
        const uint64_t v = fixed_node(xi[m * dim + d], J);
        u[(size_t)d * M + m] = v;
        cell[d] = (int64_t)(v >> (64 - G));
    }
    key[m] = (int32_t)(dim == 2 ? tile_key(cell[0], cell[1], ts, ng) : cell[0]);
    idx[m] = (int32_t)m;
}

// cs[c] = first sorted position whose key is >= c, c = 0..ncells
__global__ void cell_start_kernel(const int32_t* __restrict__ keys, int64_t M, int64_t ncells,
                                  int32_t* __restrict__ cs) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    int64_t lo = 0, hi = M;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    cs[c] = (int32_t)lo;
}

// o[i] = a[i * stride], i < n (the cell offsets at tile boundaries)
__global__ void stride_gather_kernel(const int32_t* __restrict__ a, int64_t stride, int64_t n, int32_t* __restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i * stride];
}

// positions and sqrt(mu) in sorted order, in both precisions
__global__ void gather_kernel(const int32_t* __restrict__ perm, const uint64_t* __restrict__ u,
                              const double* __restrict__ mu, int64_t M, int dim, uint64_t* __restrict__ pos64,
                              uint32_t* __restrict__ pos32, double* __restrict__ smu64, double* __restrict__ smuP64,
                              float* __restrict__ smuP32) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int64_t m = perm[q];
    for (int d = 0; d < dim; ++d) {
        const uint64_t v = u[(size_t)d * M + m];
        if (pos64) pos64[(size_t)d * M + q] = v;
        if (pos32) pos32[(size_t)d * M + q] = (uint32_t)(v >> 32);
    }
    const double s = mu ? sqrt(mu[m]) : 1.0;
    smu64[q] = s;
    if (smuP64) smuP64[q] = s;
    if (smuP32) smuP32[q] = (float)s;
}

using C64 = cx<double>;

__device__ inline C64 cmulv(C64 a, C64 b) { return mk<double>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline C64 rscale(double s, C64 a) { return mk<double>(s * a.x, s * a.y); }

// filter data of one p in one array: taps h_k (k = -p+1..p), then per edge
// (left, right) U (p x p), V (p x (2p-1)) and v1(0) (p)
template <int P> struct FilterLayout {
    static constexpr int NV = 2 * P - 1;
    static constexpr int TAPS = 0, EDGE = 2 * P, EDGE_SIZE = P * P + P * NV + P;
    static constexpr int U = 0, V = P * P, V0 = P * P + P * NV;
    static constexpr int TOTAL = 2 * P + 2 * EDGE_SIZE;
};

// channels of point x in dimension d: [L_0..L_{p-1}, D, R_0..R_{p-1}] (Haar: D)
template <int P>
__global__ void __launch_bounds__(PLAN_THREADS) basis_kernel(const double* __restrict__ xi, const int32_t* __restrict__ perm,
                                                             int64_t M, int dim, int J, const double* __restrict__ filt,
                                                             C64* __restrict__ ch64x, C64* __restrict__ ch64y,
                                                             cx<float>* __restrict__ ch32x, cx<float>* __restrict__ ch32y) {
    using L = FilterLayout<P>;
    constexpr int NB = P == 1 ? 0 : P, NCH = 2 * NB + 1, NV = L::NV;
    __shared__ double sf[L::TOTAL];
    for (int i = threadIdx.x; i < L::TOTAL; i += blockDim.x) sf[i] = filt[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * dim) return;
    const int d = (int)(t / M);
    const int64_t q = t - (int64_t)d * M;
    const double x = xi[(int64_t)perm[q] * dim + d];
    const double eta = ldexp(x, -J);
    const double* h = sf + L::TAPS;
    // product depth: 62 + ceil(log2 |eta|) levels (|eta| > 1)
    const double a = fabs(eta);
    int lg = 0;
    if (a > 1) {
        int e;
        const double mnt = frexp(a, &e);
        lg = mnt == 0.5 ? e - 1 : e;
    }
    const int Ktop = 62 + lg;
    const int K = min(Ktop - 1, 36 + lg);
    C64 wl[P > 1 ? P : 1], wr[P > 1 ? P : 1];
    if constexpr (NB > 0) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            wl[k] = mk<double>(sf[L::EDGE + L::V0 + k], 0.0);
            wr[k] = mk<double>(sf[L::EDGE + L::EDGE_SIZE + L::V0 + k], 0.0);
        }
    }
    C64 acc = mk<double>(1.0, 0.0);   // product of m0 over the levels above the current one
    for (int j = Ktop; j >= 1; --j) {
        const double zeta = ldexp(eta, -j);
        double sn, cs;
        sincos(-M_PI * zeta, &sn, &cs);
        const C64 dz = mk<double>(-2 * sn * sn, 2 * sn * cs);   // e^{-2 pi i zeta} - 1
        const C64 z = mk<double>(1.0 + dz.x, dz.y);
        if constexpr (NB > 0) {
            if (j <= K) {
                // recursion step at zeta / 2 = eta / 2^j with phi-hat(eta / 2^j) = acc
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const double* E = sf + L::EDGE + side * L::EDGE_SIZE;
                    C64* w = side == 0 ? wl : wr;
                    const C64 base = side == 0 ? z : conjc(z);
                    C64 pw = mk<double>(1.0, 0.0);
                    const int first = side == 0 ? P : P + 1;
                    for (int i = 0; i < first; ++i) pw = cmulv(pw, base);
                    C64 v2[NV];
#pragma unroll
                    for (int mi = 0; mi < NV; ++mi) {
                        v2[mi] = cmulv(acc, pw);
                        pw = cmulv(pw, base);
                    }
                    C64 w2[P];
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        C64 s = czero<double>();
#pragma unroll
                        for (int qq = 0; qq < P; ++qq) {
                            const double c = E[L::U + k * P + qq];
                            s = mk<double>(s.x + c * w[qq].x, s.y + c * w[qq].y);
                        }
                        const int last = min(NV, 2 * k + 1);   // staircase of V
#pragma unroll
                        for (int mi = 0; mi < NV; ++mi) {
                            if (mi >= last) break;
                            const double c = E[L::V + k * NV + mi];
                            s = mk<double>(s.x + c * v2[mi].x, s.y + c * v2[mi].y);
                        }
                        w2[k] = s;
                    }
#pragma unroll
                    for (int k = 0; k < P; ++k) w[k] = w2[k];
                }
            }
        }
        // m0(zeta) - 1 = sum_k h_k (z^k - 1): k = 1..p from z, k = -1..-(p-1) from conj(z)
        C64 e = dz;
        C64 m = rscale(h[1 + P - 1], e);
        for (int k = 2; k <= P; ++k) {
            e = cadd(cmulv(z, e), dz);
            m = cadd(m, rscale(h[k + P - 1], e));
        }
        if (P >= 2) {
            const C64 dc = conjc(dz), zc = conjc(z);
            e = dc;
            m = cadd(m, rscale(h[-1 + P - 1], e));
            for (int k = 2; k <= P - 1; ++k) {
                e = cadd(cmulv(zc, e), dc);
                m = cadd(m, rscale(h[-k + P - 1], e));
            }
        }
        acc = cmulv(acc, mk<double>(1.0 + m.x, m.y));
    }
    const double scale = 1.0 / sqrt(ldexp(1.0, J));
    C64 out[NCH];
    out[NB] = rscale(scale, acc);
    if constexpr (NB > 0) {
        const double r = fmod(x, 2.0);   // exact
        double sp, cp;
        sincos(M_PI * r, &sp, &cp);
        const C64 ep = mk<double>(cp, sp);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            out[c] = rscale(scale, cmulv(ep, wl[c]));
            out[NB + 1 + c] = rscale(scale, cmulv(conjc(ep), wr[c]));
        }
    }
    C64* o64 = d == 0 ? ch64x : ch64y;
    cx<float>* o32 = d == 0 ? ch32x : ch32y;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (o64) o64[(size_t)c * M + q] = out[c];
        if (o32) o32[(size_t)c * M + q] = mk<float>((float)out[c].x, (float)out[c].y);
    }
}

template <int P>
std::vector<double> filter_array(const BasisData& b) {
    using L = FilterLayout<P>;
    std::vector<double> f(L::TOTAL, 0.0);
    for (int i = 0; i < 2 * P; ++i) f[L::TAPS + i] = b.taps[i];
    if (P > 1) {
        for (int side = 0; side < 2; ++side) {
            const BoundaryEdge& E = side == 0 ? b.left : b.right;
            double* o = f.data() + L::EDGE + side * L::EDGE_SIZE;
            std::copy(E.U.begin(), E.U.end(), o + L::U);
            std::copy(E.V.begin(), E.V.end(), o + L::V);
            std::copy(E.v0.begin(), E.v0.end(), o + L::V0);
        }
    }
    return f;
}

template <int P>
hipError_t launch_basis(const Plan& P_, const double* xi, const double* filt_dev, hipStream_t s) {
    const int64_t n = P_.M * P_.dim;
    const int blocks = (int)((n + PLAN_THREADS - 1) / PLAN_THREADS);
    hipLaunchKernelGGL((basis_kernel<P>), dim3(blocks), dim3(PLAN_THREADS), 0, s, xi, P_.perm, P_.M, P_.dim, P_.J,
                       filt_dev, P_.d64.present ? P_.d64.chx : nullptr, P_.d64.present ? P_.d64.chy : nullptr,
                       P_.d32.present ? P_.d32.chx : nullptr, P_.d32.present ? P_.d32.chy : nullptr);
    return hipGetLastError();
}

template <int P>
hipError_t filter_upload(const BasisData& b, double*& dev, hipStream_t s) {
    const std::vector<double> f = filter_array<P>(b);
    GS_HIP_TRY(hipMalloc(&dev, f.size() * sizeof(double)));
    return hipMemcpyAsync(dev, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice, s);
}

template <class Ptr>
hipError_t palloc(Plan& P, Ptr*& ptr, size_t elems) {
    ptr = nullptr;
    if (elems == 0) return hipSuccess;
    void* v = nullptr;
    GS_HIP_TRY(hipMalloc(&v, elems * sizeof(Ptr)));
    ptr = static_cast<Ptr*>(v);
    P.bytes += (int64_t)(elems * sizeof(Ptr));
    return hipSuccess;
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(T*& p, size_t n) {
        void* v = nullptr;
        GS_HIP_TRY(hipMalloc(&v, std::max<size_t>(1, n) * sizeof(T)));
        ptrs.push_back(v);
        p = static_cast<T*>(v);
        return hipSuccess;
    }
};

}  // namespace

// Builds the point tables of plan P on the device: perm, cell_start,
// tile_order, and per held precision pos, chx/chy and smu, plus the solver's
// smu64 (allocated by the caller).  xi_host: M x dim frequencies, mu_host:
// M weights or nullptr.  Synchronizes `s` before returning.
hipError_t device_point_tables(Plan& P, const double* xi_host, const double* mu_host, hipStream_t s) {
    const int64_t M = P.M;
    const int dim = P.dim;
    const int nch = 2 * P.nb + 1;
    const int64_t ncells = dim == 2 ? (int64_t)P.ng * P.ng : P.ng;
    Scratch tmp;
    double *xi = nullptr, *mu = nullptr;
    GS_HIP_TRY(tmp.get(xi, (size_t)M * dim));
    GS_HIP_TRY(hipMemcpyAsync(xi, xi_host, (size_t)M * dim * sizeof(double), hipMemcpyHostToDevice, s));
    if (mu_host) {
        GS_HIP_TRY(tmp.get(mu, (size_t)M));
        GS_HIP_TRY(hipMemcpyAsync(mu, mu_host, (size_t)M * sizeof(double), hipMemcpyHostToDevice, s));
    }
    uint64_t* u = nullptr;
    int32_t *key = nullptr, *idx = nullptr, *key_sorted = nullptr;
    GS_HIP_TRY(tmp.get(u, (size_t)M * dim));
    GS_HIP_TRY(tmp.get(key, (size_t)M));
    GS_HIP_TRY(tmp.get(idx, (size_t)M));
    GS_HIP_TRY(tmp.get(key_sorted, (size_t)M));
    GS_HIP_TRY(palloc(P, P.perm, (size_t)M));
    const int blocks = (int)((M + PLAN_THREADS - 1) / PLAN_THREADS);
    hipLaunchKernelGGL(keys_kernel, dim3(blocks), dim3(PLAN_THREADS), 0, s, xi, M, dim, P.J, P.G, P.ts, P.ng, u, key,
                       idx);
    GS_HIP_TRY(hipGetLastError());
    // stable LSD radix sort of (cell key, index): points of a cell keep their input order
    const int end_bit = std::max(1, ilog2(ncells));
    size_t tbytes = 0;
    GS_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, key, key_sorted, idx, P.perm, (int)M, 0, end_bit,
                                                  s));
    void* tstore = nullptr;
    unsigned char* tb = nullptr;
    GS_HIP_TRY(tmp.get(tb, tbytes));
    tstore = tb;
    GS_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(tstore, tbytes, key, key_sorted, idx, P.perm, (int)M, 0, end_bit,
                                                  s));
    GS_HIP_TRY(palloc(P, P.cell_start, (size_t)ncells + 1));
    hipLaunchKernelGGL(cell_start_kernel, dim3((int)((ncells + PLAN_THREADS) / PLAN_THREADS)), dim3(PLAN_THREADS), 0,
                       s, key_sorted, M, ncells, P.cell_start);
    GS_HIP_TRY(hipGetLastError());
    // positions, weights and channel tables in sorted order
    if (P.d64.present) {
        GS_HIP_TRY(palloc(P, P.d64.pos, (size_t)dim * M));
        GS_HIP_TRY(palloc(P, P.d64.smu, (size_t)M));
        GS_HIP_TRY(palloc(P, P.d64.chx, (size_t)nch * M));
        if (dim == 2) GS_HIP_TRY(palloc(P, P.d64.chy, (size_t)nch * M));
    }
    if (P.d32.present) {
        GS_HIP_TRY(palloc(P, P.d32.pos, (size_t)dim * M));
        GS_HIP_TRY(palloc(P, P.d32.smu, (size_t)M));
        GS_HIP_TRY(palloc(P, P.d32.chx, (size_t)nch * M));
        if (dim == 2) GS_HIP_TRY(palloc(P, P.d32.chy, (size_t)nch * M));
    }
    hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(PLAN_THREADS), 0, s, P.perm, u, mu, M, dim,
                       P.d64.present ? P.d64.pos : nullptr, P.d32.present ? P.d32.pos : nullptr, P.smu64,
                       P.d64.present ? P.d64.smu : nullptr, P.d32.present ? P.d32.smu : nullptr);
    GS_HIP_TRY(hipGetLastError());
    const BasisData& bd = basis_data(P.p);
    double* filt = nullptr;
    hipError_t e = hipSuccess;
    switch (P.p) {
        case 1: e = filter_upload<1>(bd, filt, s); if (e == hipSuccess) e = launch_basis<1>(P, xi, filt, s); break;
        case 2: e = filter_upload<2>(bd, filt, s); if (e == hipSuccess) e = launch_basis<2>(P, xi, filt, s); break;
        case 3: e = filter_upload<3>(bd, filt, s); if (e == hipSuccess) e = launch_basis<3>(P, xi, filt, s); break;
        case 4: e = filter_upload<4>(bd, filt, s); if (e == hipSuccess) e = launch_basis<4>(P, xi, filt, s); break;
        case 5: e = filter_upload<5>(bd, filt, s); if (e == hipSuccess) e = launch_basis<5>(P, xi, filt, s); break;
        case 6: e = filter_upload<6>(bd, filt, s); if (e == hipSuccess) e = launch_basis<6>(P, xi, filt, s); break;
        case 7: e = filter_upload<7>(bd, filt, s); if (e == hipSuccess) e = launch_basis<7>(P, xi, filt, s); break;
        case 8: e = filter_upload<8>(bd, filt, s); if (e == hipSuccess) e = launch_basis<8>(P, xi, filt, s); break;
        default: e = hipErrorInvalidValue;
    }
    if (filt) tmp.ptrs.push_back(filt);
    GS_HIP_TRY(e);
    // 2D tiles in decreasing point count (stable): the tile kernels take the heaviest tiles first
    if (dim == 2 && P.ts == TILE) {
        const int64_t nt = (int64_t)(P.ng / P.ts) * (P.ng / P.ts), tc = (int64_t)P.ts * P.ts;
        int32_t* tb_dev = nullptr;
        GS_HIP_TRY(tmp.get(tb_dev, (size_t)nt + 1));
        hipLaunchKernelGGL(stride_gather_kernel, dim3((int)((nt + PLAN_THREADS) / PLAN_THREADS)), dim3(PLAN_THREADS), 0,
                           s, P.cell_start, tc, nt + 1, tb_dev);
        GS_HIP_TRY(hipGetLastError());
        std::vector<int32_t> bounds(nt + 1);
        GS_HIP_TRY(hipMemcpyAsync(bounds.data(), tb_dev, (nt + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GS_HIP_TRY(hipStreamSynchronize(s));
        std::vector<int32_t> order(nt);
        for (int64_t t = 0; t < nt; ++t) order[t] = (int32_t)t;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return bounds[a + 1] - bounds[a] > bounds[b + 1] - bounds[b];
        });
        GS_HIP_TRY(palloc(P, P.tile_order, (size_t)nt));
        GS_HIP_TRY(hipMemcpyAsync(P.tile_order, order.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    return hipStreamSynchronize(s);
}

}  // namespace gs
