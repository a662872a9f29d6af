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

// in-place decimation-in-time FFT on CB transforms buf[c*n + i], input in
// bit-reversed order.  Two radix-2 stages are fused into one radix-4 pass
// (one LDS round trip and one barrier per pair of stages); an odd stage count
// ends with a radix-2 pass.  tw[m] = e^{-2 pi i m / ng}; twstride = ng / n.
template <class T, int DIR>
__device__ inline void lds_fft(cx<T>* buf, int n, int logn, int CB, const cx<T>* __restrict__ tw, int twstride) {
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);          // half length of the first fused stage
        const int nq = CB * (n >> 2);        // radix-4 butterflies
        __syncthreads();
        for (int i = threadIdx.x; i < nq; i += blockDim.x) {
            const int c = i >> (logn - 2);
            const int j = i & ((n >> 2) - 1);
            const int k = j & (h - 1);
            const int grp = j >> (s - 1);
            const int a = c * n + grp * 4 * h + k;
            cx<T> w1 = tw[(k << (logn - s)) * twstride];          // e^{-2 pi i k / 2h}
            cx<T> w2 = tw[(k << (logn - s - 1)) * twstride];      // e^{-2 pi i k / 4h}
            if (DIR > 0) { w1.y = -w1.y; w2.y = -w2.y; }
            const cx<T> x0 = buf[a], x1 = buf[a + h], x2 = buf[a + 2 * h], x3 = buf[a + 3 * h];
            const cx<T> t1 = cmul(x1, w1), t3 = cmul(x3, w1);
            const cx<T> y0 = cadd(x0, t1), y1 = csub(x0, t1), y2 = cadd(x2, t3), y3 = csub(x2, t3);
            const cx<T> u2 = cmul(y2, w2);
            // w3 = w2 * e^{-+ i pi/2}: multiply by -i (forward) or +i (adjoint)
            cx<T> u3 = cmul(y3, w2);
            u3 = (DIR > 0) ? mk<T>(-u3.y, u3.x) : mk<T>(u3.y, -u3.x);
            buf[a] = cadd(y0, u2);
            buf[a + 2 * h] = csub(y0, u2);
            buf[a + h] = cadd(y1, u3);
            buf[a + 3 * h] = csub(y1, u3);
        }
    }
    if (s == logn) {                          // remaining radix-2 stage
        const int half = 1 << (s - 1);
        const int nbf = CB * (n >> 1);
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

// columns per workgroup for strided (column) passes: keep LDS <= 32 KB
template <class T>
inline int col_batch(int n) {
    int cb = (int)(32768 / ((size_t)n * sizeof(cx<T>)));
    if (cb > 16) cb = 16;
    if (cb < 1) cb = 1;
    return cb;
}

}  // namespace gs
