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

template <class T, class Op>
struct FftArgs {
    Op op;
    const cx<T>* tw;
    double* nsq;   // per-workgroup sums of the stored |value|^2, for ops whose store returns it
};


template <class T, int DIR, class Op>
__device__ __forceinline__ void fft_kernel_body(const FftArgs<T, Op>& a, int n, int logn, int CB, int twstride, int ntrans) {
    const Op& op = a.op;
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int t0 = blockIdx.x * CB;
    for (int e = threadIdx.x; e < CB * n; e += blockDim.x) {
        const int c = e % CB, i = e / CB;
        const int t = t0 + c;
        buf[c * n + bitrev(i, logn)] = (t < ntrans) ? op.load(t, i) : czero<T>();
    }
    lds_fft<T, DIR>(buf, n, logn, CB, a.tw, twstride);
    using R = decltype(op.store(0, 0, czero<T>()));
    if constexpr (std::is_same<R, double>::value) {
        double acc = 0;
        for (int e = threadIdx.x; e < CB * n; e += blockDim.x) {
            const int c = e % CB, k = e / CB;
            const int t = t0 + c;
            if (t < ntrans) acc += op.store(t, k, buf[c * n + k]);
        }
        if (a.nsq) {
            __shared__ double sh[4];
            const double v = wg_sum(acc, sh);
            if (threadIdx.x == 0) a.nsq[blockIdx.x] = v;
        }
    } else {
        for (int e = threadIdx.x; e < CB * n; e += blockDim.x) {
            const int c = e % CB, k = e / CB;
            const int t = t0 + c;
            if (t < ntrans) op.store(t, k, buf[c * n + k]);
        }
    }
}

template <class T, int DIR, class Op, bool BATCH>
__global__ void __launch_bounds__(256) fft_kernel(FftArgs<T, Op> one, const FftArgs<T, Op>* __restrict__ many, int n, int logn,
                                                 int CB, int twstride, int ntrans) {
    if constexpr (BATCH) {
        const FftArgs<T, Op> a = kernel_args<true>(one, many);
        fft_kernel_body<T, DIR, Op>(a, n, logn, CB, twstride, ntrans);
    } else {
        fft_kernel_body<T, DIR, Op>(one, n, logn, CB, twstride, ntrans);
    }
}

template <class T, int DIR, class Op>
inline hipError_t launch_fft(const Op& op, int ntrans, int n, int CB, const cx<T>* tw, int ng, hipStream_t s,
                             double* nsq = nullptr) {
    if (ntrans <= 0) return hipSuccess;
    const int logn = ilog2(n);
    const int blocks = (ntrans + CB - 1) / CB;
    const size_t sh = (size_t)CB * n * sizeof(cx<T>);
    int threads = CB * n / 2;
    threads = threads < 64 ? 64 : (threads > 256 ? 256 : threads);
    using A = FftArgs<T, Op>;
    return launch_site(A{op, tw, nsq}, [&](const A& one, const A* many, int count) {
        if (many) hipLaunchKernelGGL((fft_kernel<T, DIR, Op, true>), dim3(blocks, count), dim3(threads), sh, s, one, many, n, logn, CB,
                           ng / n, ntrans);
        else hipLaunchKernelGGL((fft_kernel<T, DIR, Op, false>), dim3(blocks, count), dim3(threads), sh, s, one, many, n, logn, CB,
                           ng / n, ntrans);
        return hipGetLastError();
    });
}

// ------------------------------------------------------------ register FFTs
// Column transforms of an ng x ng grid with ng = R1 * R2, two passes over HBM.
// A thread holds one R-point transform in registers; a wavefront covers 64
// adjacent columns, so every load and store is a contiguous row segment.
//   pass 1, thread (col, n2): Y[k1] = W_ng^(n2 k1) sum_n1 x[R2 n1 + n2] W_R1^(n1 k1),
//     written back to row R2 k1 + n2;
//   pass 2, thread (col, k1): X[k1 + R1 k2] = sum_n2 Y[R2 k1 + n2] W_R2^(n2 k2),
//     written to row R2 k1 + k2.
// Both passes are in place; frequency row k ends in row R2 (k mod R1) + k / R1.
template <int R>
__host__ __device__ constexpr int brev_ct(int i) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// in-register R-point DFT, natural order in and out; tw[m * tstep] = e^{-2 pi i m / R}
template <class T, int R, int DIR>
__device__ inline void reg_fft(cx<T>* v, const cx<T>* tw, int tstep) {
    cx<T> a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = v[brev_ct<R>(i)];
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int k = 0; k < h; ++k) {
            cx<T> w = tw[k * (R / (2 * h)) * tstep];
            if (DIR > 0) w.y = -w.y;
#pragma unroll
            for (int g = 0; g < R; g += 2 * h) {
                const cx<T> u = a[g + k];
                const cx<T> t = k == 0 ? a[g + k + h] : cmul(a[g + k + h], w);
                a[g + k] = cadd(u, t);
                a[g + k + h] = csub(u, t);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = a[i];
}

// rows whose frequency lies in [-(N/2) + nb, N/2 - nb): the interior of the 2D grid
__device__ inline bool grid_row_active(int q, int ng, int N, int nb) {
    const int k = q < (ng >> 1) ? q : q - ng;
    return k >= -(N >> 1) + nb && k < (N >> 1) - nb;
}

// input of a column pass 1: element (row q, column c) of the grid, inactive rows
// read as zero when prune is set (forward)
template <class T>
struct GridLoad {
    const cx<T>* grid;
    int L, N, nb, prune;
    __device__ cx<T> operator()(int q, int col) const {
        return (prune && !grid_row_active(q, L, N, nb)) ? czero<T>() : grid[(size_t)q * L + col];
    }
};

template <class T, class Load>
struct ColArgs {
    Load ld;
    cx<T>* grid;
    const cx<T>* tw;
};

template <class T, int R1, int R2, int DIR, class Load>
__device__ __forceinline__ void colfft_pass1_body(const ColArgs<T, Load>& a) {
    const Load& ld = a.ld;
    cx<T>* __restrict__ grid = a.grid;
    constexpr int L = R1 * R2;
    __shared__ cx<T> stw[L];
    for (int e = threadIdx.x; e < L; e += 256) stw[e] = a.tw[e];
    __syncthreads();
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int n2 = blockIdx.z * 4 + (threadIdx.x >> 6);
    cx<T> v[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) v[n1] = ld(R2 * n1 + n2, col);
    reg_fft<T, R1, DIR>(v, stw, L / R1);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        cx<T> w = stw[(n2 * k1) & (L - 1)];
        if (DIR > 0) w.y = -w.y;
        grid[(size_t)(R2 * k1 + n2) * L + col] = cmul(v[k1], w);
    }
}

template <class T, int R1, int R2, int DIR, class Load, bool BATCH>
__global__ void __launch_bounds__(256) colfft_pass1(ColArgs<T, Load> one, const ColArgs<T, Load>* __restrict__ many) {
    if constexpr (BATCH) {
        const ColArgs<T, Load> a = kernel_args<true>(one, many);
        colfft_pass1_body<T, R1, R2, DIR, Load>(a);
    } else {
        colfft_pass1_body<T, R1, R2, DIR, Load>(one);
    }
}

template <class T>
struct Col2Args {
    cx<T>* grid;
    const cx<T>* tw;
};

template <class T, int R1, int R2, int DIR>
__device__ __forceinline__ void colfft_pass2_body(const Col2Args<T>& a, int N, int nb, int prune_out) {
    cx<T>* __restrict__ grid = a.grid;
    constexpr int L = R1 * R2;
    __shared__ cx<T> stw[L];
    for (int e = threadIdx.x; e < L; e += 256) stw[e] = a.tw[e];
    __syncthreads();
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int k1 = blockIdx.z * 4 + (threadIdx.x >> 6);
    cx<T> v[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) v[n2] = grid[(size_t)(R2 * k1 + n2) * L + col];
    reg_fft<T, R2, DIR>(v, stw, L / R2);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
        if (prune_out && !grid_row_active(k1 + R1 * k2, L, N, nb)) continue;
        grid[(size_t)(R2 * k1 + k2) * L + col] = v[k2];
    }
}

template <class T, int R1, int R2, int DIR, bool BATCH>
__global__ void __launch_bounds__(256) colfft_pass2(Col2Args<T> one, const Col2Args<T>* __restrict__ many, int N, int nb,
                                                    int prune_out) {
    if constexpr (BATCH) {
        const Col2Args<T> a = kernel_args<true>(one, many);
        colfft_pass2_body<T, R1, R2, DIR>(a, N, nb, prune_out);
    } else {
        colfft_pass2_body<T, R1, R2, DIR>(one, N, nb, prune_out);
    }
}

// both passes; Load supplies the input of pass 1 (prune_out: inactive output rows are not stored)
template <class T, int R1, int R2, int DIR, class Load>
inline hipError_t launch_colfft(const Load& ld, cx<T>* grid, const cx<T>* tw, int N, int nb, int prune_out,
                                hipStream_t s) {
    constexpr int L = R1 * R2;
    using A1 = ColArgs<T, Load>;
    GS_HIP_TRY(launch_site(A1{ld, grid, tw}, [&](const A1& one, const A1* many, int count) {
        if (many) hipLaunchKernelGGL((colfft_pass1<T, R1, R2, DIR, Load, true>), dim3(L / 64, count, R2 / 4), dim3(256), 0, s, one,
                           many);
        else hipLaunchKernelGGL((colfft_pass1<T, R1, R2, DIR, Load, false>), dim3(L / 64, count, R2 / 4), dim3(256), 0, s, one,
                           many);
        return hipGetLastError();
    }));
    using A2 = Col2Args<T>;
    return launch_site(A2{grid, tw}, [&](const A2& one, const A2* many, int count) {
        if (many) hipLaunchKernelGGL((colfft_pass2<T, R1, R2, DIR, true>), dim3(L / 64, count, R1 / 4), dim3(256), 0, s, one, many, N,
                           nb, prune_out);
        else hipLaunchKernelGGL((colfft_pass2<T, R1, R2, DIR, false>), dim3(L / 64, count, R1 / 4), dim3(256), 0, s, one, many, N,
                           nb, prune_out);
        return hipGetLastError();
    });
}

// the column split of Plan::cr1 for grids of side ng; LoadF(L) builds the pass-1 input
template <class T, int DIR, class LoadF>
inline hipError_t launch_colfft_split(int cr1, int ng, const LoadF& mk, cx<T>* grid, const cx<T>* tw, int N, int nb,
                                      int prune_out, hipStream_t s) {
    if (ng == 1024 && cr1 == 32) return launch_colfft<T, 32, 32, DIR>(mk(1024), grid, tw, N, nb, prune_out, s);
    if (ng == 512 && cr1 == 32) return launch_colfft<T, 32, 16, DIR>(mk(512), grid, tw, N, nb, prune_out, s);
    if (ng == 256 && cr1 == 16) return launch_colfft<T, 16, 16, DIR>(mk(256), grid, tw, N, nb, prune_out, s);
    return hipErrorInvalidValue;
}

// a pair of transform sets in one launch: transforms [0, na) of a, then those of b
template <class T, class A, class B>
struct OpJoin {
    A a;
    B b;
    int na;
    __device__ cx<T> load(int t, int i) const { return t < na ? a.load(t, i) : b.load(t - na, i); }
    __device__ auto store(int t, int k, cx<T> v) const {
        if (t < na) return a.store(t, k, v);
        return b.store(t - na, k, v);
    }
};

// columns per workgroup for strided (column) passes: keep LDS <= 32 KB
template <class T>
inline int col_batch(int n) {
    int cb = (int)(32768 / ((size_t)n * sizeof(cx<T>)));
    if (cb > 16) cb = 16;
    if (cb < 1) cb = 1;
    return cb;
}

}  // namespace gs
