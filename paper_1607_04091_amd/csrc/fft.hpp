// Power-of-two complex FFTs in LDS for the NFFT grids (gfx950).
//
// A workgroup loads CB transforms of length n through a load functor (which
// fuses deapodization, zero padding or cropping), runs an in-place radix-2
// decimation-in-time transform in LDS and writes through a store functor.
// Forward sign (DIR = -1): g_l = sum_k g^_k e^{-2 pi i k l / n}; DIR = +1 is
// the adjoint (unnormalized).  Transform sizes above FFT_MAX_LDS use a
// four-step split n = n1 * n2 with an intermediate twiddle multiplication.
#pragma once

#include "common.hpp"

namespace gs {

__device__ inline int bitrev(int i, int logn) { return logn ? (int)(__brev((unsigned)i) >> (32 - logn)) : 0; }

// in-place radix-2 DIT on CB transforms buf[c*n + i], input in bit-reversed order.
// tw[m] = e^{-2 pi i m / ng}; twstride = ng / n.
template <class T, int DIR>
__device__ inline void lds_fft(cx<T>* buf, int n, int logn, int CB, const cx<T>* __restrict__ tw, int twstride) {
    const int nbf = CB * (n >> 1);
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        __syncthreads();
        for (int i = threadIdx.x; i < nbf; i += blockDim.x) {
            const int c = i >> (logn - 1);
            const int j = i & ((n >> 1) - 1);
            const int k = j & (half - 1);
            const int grp = j >> (s - 1);
            const int a = c * n + (grp << s) + k;
            const int b = a + half;
            cx<T> w = tw[(k << (logn - s)) * twstride];
            if (DIR > 0) w.y = -w.y;
            const cx<T> u = buf[a];
            const cx<T> v = cmul(buf[b], w);
            buf[a] = cadd(u, v);
            buf[b] = csub(u, v);
        }
    }
    __syncthreads();
}

template <class T, int DIR, class Op>
__global__ void __launch_bounds__(256) fft_kernel(Op op, const cx<T>* __restrict__ tw, int n, int logn, int CB,
                                                 int twstride, int ntrans) {
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int t0 = blockIdx.x * CB;
    for (int e = threadIdx.x; e < CB * n; e += blockDim.x) {
        const int c = e % CB, i = e / CB;
        const int t = t0 + c;
        buf[c * n + bitrev(i, logn)] = (t < ntrans) ? op.load(t, i) : czero<T>();
    }
    lds_fft<T, DIR>(buf, n, logn, CB, tw, twstride);
    for (int e = threadIdx.x; e < CB * n; e += blockDim.x) {
        const int c = e % CB, k = e / CB;
        const int t = t0 + c;
        if (t < ntrans) op.store(t, k, buf[c * n + k]);
    }
}

template <class T, int DIR, class Op>
inline hipError_t launch_fft(const Op& op, int ntrans, int n, int CB, const cx<T>* tw, int ng, hipStream_t s) {
    if (ntrans <= 0) return hipSuccess;
    const int logn = ilog2(n);
    const int blocks = (ntrans + CB - 1) / CB;
    const size_t sh = (size_t)CB * n * sizeof(cx<T>);
    int threads = CB * n / 2;
    threads = threads < 64 ? 64 : (threads > 256 ? 256 : threads);
    hipLaunchKernelGGL((fft_kernel<T, DIR, Op>), dim3(blocks), dim3(threads), sh, s, op, tw, n, logn, CB, ng / n,
                       ntrans);
    return hipGetLastError();
}

// columns per workgroup for strided (column) passes: keep LDS <= 64 KB
template <class T>
inline int col_batch(int n) {
    int cb = (int)(65536 / ((size_t)n * sizeof(cx<T>)));
    if (cb > 16) cb = 16;
    if (cb < 1) cb = 1;
    return cb;
}

}  // namespace gs
