// Device-resident CGLS for the weighted least-squares problem
// argmin ||W^{1/2}(T x - y)|| (Sec. 2 eq. least_squares; Sec. 4.1 eq.
// weighted_least_squares; the paper's "conjugate gradient procedure").
//
// A = W^{1/2} T, b = W^{1/2} y.  Iteration (CG on the normal equations):
//   q = A p; delta = ||q||^2; alpha = gamma/delta; x += alpha p; r -= alpha q;
//   s = A^H r; gamma' = ||s||^2; p = s + (gamma'/gamma) p; gamma = gamma'.
// Stop when sqrt(gamma) <= tol * ||A^H b||.  All vectors, reductions and
// scalars are FP64 and stay on the device; the applies run in the plan's
// precision.  Reductions are two-stage with a fixed block count and a fixed
// summation order, so results are bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "prof.hpp"

namespace gs {

constexpr int RB = 512;      // reduction blocks (fixed -> deterministic)
constexpr int RT = 256;      // threads per reduction block

// S_GMIN: smallest gamma of the current run; S_GROW: stall factor (0 = off);
// S_STALL: the run stopped because gamma rose above S_GROW * S_GMIN.
// The four scalars the iteration advances (gamma, done, break, gmin) have two
// copies: workgroup 0 of update_p writes the first (the step of the
// iteration) while its other workgroups read only the second, which workgroup
// 0 of update_xr refreshes from the first while its workgroups read only the
// first.  No workgroup reads a slot its own kernel writes.
enum Scal {
    S_GAMMA = 0, S_DELTA, S_ALPHA, S_REF, S_TOL2, S_DONE, S_BREAK, S_ITER, S_REF64, S_GMIN, S_GROW, S_STALL,
    S_GAMMA_B, S_DONE_B, S_BREAK_B, S_GMIN_B,
    S_NSCAL = 16
};
static_assert(S_GMIN_B < S_NSCAL, "scalar slots");

template <class T> __device__ inline cx<double> to64(cx<T> v) { return mk<double>((double)v.x, (double)v.y); }

__device__ inline double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// sum of n partials, same order in every block
__device__ inline double sum_partials(const double* __restrict__ red, int n, double* sh) {
    double v = 0;
    for (int i = threadIdx.x; i < n; i += RT) v += red[i];
    return block_sum(v, sh);
}

template <class T>
struct Norm2Args {
    const cx<T>* v;
    int64_t n;
    double* red;
};

template <class T>
__device__ __forceinline__ void norm2_partial_kernel_body(const Norm2Args<T>& A) {
    const cx<T>* __restrict__ v = A.v;
    const int64_t n = A.n;
    double* __restrict__ red = A.red;
    __shared__ double sh[RT];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)RB * RT) {
        const cx<double> a = to64(v[i]);
        acc += a.x * a.x + a.y * a.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

template <class T, bool BATCH>
__global__ void __launch_bounds__(RT) norm2_partial_kernel(Norm2Args<T> one, const Norm2Args<T>* __restrict__ many) {
    if constexpr (BATCH) {
        const Norm2Args<T> a = kernel_args<true>(one, many);
        norm2_partial_kernel_body<T>(a);
    } else {
        norm2_partial_kernel_body<T>(one);
    }
}

// b = sqrt(mu) * y[perm]; r = b (x0 = 0) ; optional FP32 copy of r
template <class Tr>
__global__ void init_b_kernel(const cx<double>* __restrict__ y, const int32_t* __restrict__ perm,
                              const double* __restrict__ smu, int64_t M, cx<double>* __restrict__ b,
                              cx<double>* __restrict__ r, cx<Tr>* __restrict__ rT) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const cx<double> v = cscale(y[perm[m]], smu[m]);
    b[m] = v;
    r[m] = v;
    if (rT) rT[m] = mk<Tr>((Tr)v.x, (Tr)v.y);
}

// r = b - q  (q = A x in apply precision), optional FP32 copy
template <class T, class Tr>
__global__ void residual_kernel(const cx<double>* __restrict__ b, const cx<T>* __restrict__ q, int64_t M,
                                cx<double>* __restrict__ r, cx<Tr>* __restrict__ rT) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const cx<double> v = csub(b[m], to64(q[m]));
    r[m] = v;
    if (rT) rT[m] = mk<Tr>((Tr)v.x, (Tr)v.y);
}

template <class T>
__global__ void convert_kernel(const cx<double>* __restrict__ a, cx<T>* __restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = mk<T>((T)a[i].x, (T)a[i].y);
}

template <class T>
__global__ void zero_kernel(cx<T>* __restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = czero<T>();
}

// p = s (in FP64 and, if FP32 applies, FP32); gamma = ||s||^2 is reduced separately
template <class T, class Tp>
__global__ void init_p_kernel(const cx<T>* __restrict__ s, cx<double>* __restrict__ p, cx<Tp>* __restrict__ pT,
                              int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cx<double> v = to64(s[i]);
    p[i] = v;
    if (pT) pT[i] = mk<Tp>((Tp)v.x, (Tp)v.y);
}

// scalar setup after the first A^H r: gamma, ref, done flag
__global__ void start_scalars_kernel(double* __restrict__ scal, const double* __restrict__ red, int nred, int set_ref,
                                     double* __restrict__ hist, int hist_len) {
    __shared__ double sh[RT];
    const double g = sum_partials(red, nred, sh);
    if (threadIdx.x == 0) {
        scal[S_GAMMA] = g;
        if (set_ref) scal[S_REF] = sqrt(g);
        scal[S_ITER] = 0;
        scal[S_BREAK] = 0;
        scal[S_GMIN] = g;
        scal[S_STALL] = 0;
        const double ref = scal[S_REF];
        scal[S_DONE] = (ref == 0.0 || g <= scal[S_TOL2] * ref * ref) ? 1.0 : 0.0;
        if (hist && hist_len > 0) hist[0] = ref > 0 ? sqrt(g) / ref : 0.0;
    }
}

__global__ void set_ref64_kernel(double* __restrict__ scal, const double* __restrict__ red) {
    __shared__ double sh[RT];
    const double g = sum_partials(red, RB, sh);
    if (threadIdx.x == 0) scal[S_REF64] = sqrt(g);
}

// x += alpha p ; r -= alpha q ; alpha = gamma / ||q||^2
template <class T, class Tr>
struct UpdateXrArgs {
    double* scal;
    const double* red;
    int nred;
    cx<double>* x;
    const cx<double>* p;
    int64_t nx;
    cx<double>* r;
    const cx<T>* q;
    cx<Tr>* rT;
    int64_t M;
};

template <class T, class Tr>
__device__ __forceinline__ void update_xr_kernel_body(const UpdateXrArgs<T, Tr>& A) {
    double* __restrict__ scal = A.scal;
    const double* __restrict__ red = A.red;
    cx<double>* __restrict__ x = A.x;
    const cx<double>* __restrict__ p = A.p;
    const int64_t nx = A.nx;
    cx<double>* __restrict__ r = A.r;
    const cx<T>* __restrict__ q = A.q;
    cx<Tr>* __restrict__ rT = A.rT;
    const int64_t M = A.M;
    __shared__ double sh[RT];
    const double delta = sum_partials(red, A.nred, sh);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (lead) {
        scal[S_GAMMA_B] = scal[S_GAMMA];
        scal[S_DONE_B] = scal[S_DONE];
        scal[S_BREAK_B] = scal[S_BREAK];
        scal[S_GMIN_B] = scal[S_GMIN];
    }
    if (scal[S_DONE] != 0.0 || scal[S_BREAK] != 0.0) return;
    const double alpha = scal[S_GAMMA] / delta;
    if (!(delta > 0.0) || !isfinite(delta) || !isfinite(alpha)) {
        if (lead) scal[S_BREAK_B] = 1.0;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_DELTA] = delta;
        scal[S_ALPHA] = alpha;
    }
    const int64_t total = nx + M;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < total; i += (int64_t)gridDim.x * RT) {
        if (i < nx) {
            const cx<double> pv = p[i];
            cx<double> xv = x[i];
            xv.x += alpha * pv.x;
            xv.y += alpha * pv.y;
            x[i] = xv;
        } else {
            const int64_t m = i - nx;
            const cx<double> qv = to64(q[m]);
            cx<double> rv = r[m];
            rv.x -= alpha * qv.x;
            rv.y -= alpha * qv.y;
            r[m] = rv;
            if (rT) rT[m] = mk<Tr>((Tr)rv.x, (Tr)rv.y);
        }
    }
}

template <class T, class Tr, bool BATCH>
__global__ void __launch_bounds__(RT) update_xr_kernel(UpdateXrArgs<T, Tr> one, const UpdateXrArgs<T, Tr>* __restrict__ many) {
    if constexpr (BATCH) {
        const UpdateXrArgs<T, Tr> a = kernel_args<true>(one, many);
        update_xr_kernel_body<T, Tr>(a);
    } else {
        update_xr_kernel_body<T, Tr>(one);
    }
}

// p = s + beta p, beta = ||s||^2 / gamma.  With xbest (reduced-precision
// recurrences), x is also copied there whenever its normal residual ||s||^2
// is the smallest of the run, so that a recurrence stopped past its accuracy
// floor can return its best iterate.  Workgroup 0 then takes the step of the
// scalars: gamma = ||s||^2, iteration count, history, convergence test.
template <class T, class Tp>
struct UpdatePArgs {
    double* scal;
    const double* red;
    int nred;
    double* hist;
    int hist_len;
    cx<double>* p;
    const cx<T>* s;
    cx<Tp>* pT;
    int64_t nx;
    const cx<double>* x;
    cx<double>* xbest;
};

template <class T, class Tp>
__device__ __forceinline__ void update_p_kernel_body(const UpdatePArgs<T, Tp>& A) {
    double* __restrict__ scal = A.scal;
    const double* __restrict__ red = A.red;
    cx<double>* __restrict__ p = A.p;
    const cx<T>* __restrict__ s = A.s;
    cx<Tp>* __restrict__ pT = A.pT;
    const int64_t nx = A.nx;
    const cx<double>* __restrict__ x = A.x;
    cx<double>* __restrict__ xbest = A.xbest;
    __shared__ double sh[RT];
    const double gnew = sum_partials(red, A.nred, sh);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (scal[S_DONE_B] != 0.0) return;
    if (scal[S_BREAK_B] != 0.0) {
        if (lead) {
            scal[S_BREAK] = 1.0;
            scal[S_DONE] = 1.0;
        }
        return;
    }
    const double gmin = scal[S_GMIN_B];
    const double beta = gnew / scal[S_GAMMA_B];
    const bool keep = xbest && gnew < gmin;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < nx; i += (int64_t)gridDim.x * RT) {
        const cx<double> sv = to64(s[i]);
        cx<double> pv = p[i];
        pv.x = sv.x + beta * pv.x;
        pv.y = sv.y + beta * pv.y;
        p[i] = pv;
        if (pT) pT[i] = mk<Tp>((Tp)pv.x, (Tp)pv.y);
        if (keep) xbest[i] = x[i];
    }
    if (!lead) return;
    scal[S_GAMMA] = gnew;
    const double it = scal[S_ITER] + 1.0;
    scal[S_ITER] = it;
    const double ref = scal[S_REF];
    if (A.hist && (int)it < A.hist_len) A.hist[(int)it] = sqrt(gnew) / ref;
    if (gnew <= scal[S_TOL2] * ref * ref) {
        scal[S_DONE] = 1.0;
    } else if (scal[S_GROW] > 0.0 && !(gnew <= scal[S_GROW] * gmin)) {
        // reduced-precision recurrence past its accuracy floor: stop it here
        scal[S_STALL] = 1.0;
        scal[S_BREAK] = 1.0;
        scal[S_DONE] = 1.0;
    }
    scal[S_GMIN] = fmin(gmin, gnew);
}

template <class T, class Tp, bool BATCH>
__global__ void __launch_bounds__(RT) update_p_kernel(UpdatePArgs<T, Tp> one, const UpdatePArgs<T, Tp>* __restrict__ many) {
    if constexpr (BATCH) {
        const UpdatePArgs<T, Tp> a = kernel_args<true>(one, many);
        update_p_kernel_body<T, Tp>(a);
    } else {
        update_p_kernel_body<T, Tp>(one);
    }
}

__global__ void copy_kernel(const cx<double>* __restrict__ a, cx<double>* __restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i];
}

__global__ void set_scalar_kernel(double* __restrict__ scal, int idx, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scal[idx] = v;
}

inline int nb256(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

template <class T>
hipError_t launch_norm2(const cx<T>* v, int64_t n, double* red, hipStream_t st) {
    using A = Norm2Args<T>;
    return launch_site(A{v, n, red}, [&](const A& one, const A* many, int count) {
        if (many) hipLaunchKernelGGL((norm2_partial_kernel<T, true>), dim3(RB, count), dim3(RT), 0, st, one, many);
        else hipLaunchKernelGGL((norm2_partial_kernel<T, false>), dim3(RB, count), dim3(RT), 0, st, one, many);
        return hipGetLastError();
    });
}

hipError_t solver_alloc(Plan& P) {
    auto alloc = [&](auto*& ptr, size_t n) -> hipError_t {
        void* v = nullptr;
        hipError_t e = hipMalloc(&v, n * sizeof(*ptr));
        if (e != hipSuccess) return e;
        ptr = static_cast<std::remove_reference_t<decltype(ptr)>>(v);
        P.bytes += (int64_t)(n * sizeof(*ptr));
        return hipSuccess;
    };
    const size_t M = P.M, nx = P.dim == 2 ? (size_t)P.N * P.N : (size_t)P.N;
    GS_HIP_TRY(alloc(P.smu64, M));
    GS_HIP_TRY(alloc(P.b, M));
    GS_HIP_TRY(alloc(P.r, M));
    GS_HIP_TRY(alloc(P.q, M));
    GS_HIP_TRY(alloc(P.ps, nx));
    GS_HIP_TRY(alloc(P.ss, nx));
    if (P.d32.present) {
        GS_HIP_TRY(alloc(P.xbest, nx));
        GS_HIP_TRY(alloc(P.q32, M));
        GS_HIP_TRY(alloc(P.r32, M));
        GS_HIP_TRY(alloc(P.p32, nx));
        GS_HIP_TRY(alloc(P.s32, nx));
    }
    P.red_blocks = std::max(RB, norm_parts_TH(P));
    GS_HIP_TRY(alloc(P.red, (size_t)P.red_blocks));
    GS_HIP_TRY(alloc(P.scal, (size_t)S_NSCAL));
    P.hist_len = 1 << 16;
    GS_HIP_TRY(alloc(P.hist, (size_t)P.hist_len));
    void* hs = nullptr;
    GS_HIP_TRY(hipHostMalloc(&hs, S_NSCAL * sizeof(double), hipHostMallocDefault));
    P.host_scal = static_cast<double*>(hs);
    return hipSuccess;
}

// ------------------------------------------------------------------ solver loop

template <class T>
struct Ops;

// FP64 applies: operands are the FP64 solver vectors themselves
template <>
struct Ops<double> {
    const Plan& P;
    cx<double>* qa() const { return P.q; }
    cx<double>* sa() const { return P.ss; }
    cx<double>* ra() const { return P.r; }
    cx<double>* pa() const { return P.ps; }
    cx<double>* rcopy() const { return nullptr; }
    cx<double>* pcopy() const { return nullptr; }
    cx<double>* xbest() const { return nullptr; }   // FP64 recurrences do not stall
};
template <>
struct Ops<float> {
    const Plan& P;
    cx<float>* qa() const { return P.q32; }
    cx<float>* sa() const { return P.s32; }
    cx<float>* ra() const { return P.r32; }
    cx<float>* pa() const { return P.p32; }
    cx<float>* rcopy() const { return P.r32; }
    cx<float>* pcopy() const { return P.p32; }
    cx<double>* xbest() const { return P.xbest; }
};

constexpr int AFLAGS = GS_WEIGHTED | GS_SORTED;

// q = A p with ||q||^2 as RB partial sums in P.red, and s = A^H r with
// ||s||^2 as partial sums in P.red: written by the adjoint's last launch
// where its path provides them, else by a separate reduction.  Returns the
// number of partials through nred.
template <class T>
hipError_t apply_T_norm(const Plan& P, const cx<T>* x, cx<T>* y, hipStream_t st, int& nred) {
    GS_HIP_TRY(launch_apply_T<T>(P, x, y, AFLAGS, st));
    GS_HIP_TRY(launch_norm2<T>(y, P.M, P.red, st));
    nred = RB;
    return hipSuccess;
}
template <class T>
hipError_t apply_TH_norm(const Plan& P, const cx<T>* u, cx<T>* x, hipStream_t st, int& nred) {
    const int n = norm_parts_TH(P);
    GS_HIP_TRY(launch_apply_TH<T>(P, u, x, AFLAGS, st, nullptr, n ? P.red : nullptr));
    if (!n) GS_HIP_TRY(launch_norm2<T>(x, P.dim == 2 ? (int64_t)P.N * P.N : P.N, P.red, st));
    nred = n ? n : RB;
    return hipSuccess;
}

// Starts CGLS from x (already on device, FP64) given r = b - A x in P.r (and
// its apply-precision copy).  Computes s = A^H r, gamma, p = s.
template <class T>
hipError_t cgls_start(const Plan& P, const cx<double>* x, hipStream_t st, int set_ref, double* hist, int hist_len) {
    Ops<T> o{P};
    const int64_t nx = P.dim == 2 ? (int64_t)P.N * P.N : P.N;
    if (o.xbest()) hipLaunchKernelGGL(copy_kernel, dim3(nb256(nx)), dim3(256), 0, st, x, o.xbest(), nx);
    int nred = 0;
    GS_HIP_TRY(apply_TH_norm<T>(P, o.ra(), o.sa(), st, nred));
    hipLaunchKernelGGL((init_p_kernel<T, T>), dim3(nb256(nx)), dim3(256), 0, st, o.sa(), P.ps, o.pcopy(), nx);
    hipLaunchKernelGGL(start_scalars_kernel, dim3(1), dim3(RT), 0, st, P.scal, P.red, nred, set_ref, hist, hist_len);
    return hipGetLastError();
}

template <class T>
hipError_t cgls_iteration(const Plan& P, cx<double>* x, hipStream_t st, double* hist, int hist_len) {
    Ops<T> o{P};
    const int64_t nx = P.dim == 2 ? (int64_t)P.N * P.N : P.N;
    const int64_t M = P.M;
    int nq = 0, ns = 0;
    GS_HIP_TRY(apply_T_norm<T>(P, o.pa(), o.qa(), st, nq));
    using AX = UpdateXrArgs<T, T>;
    GS_HIP_TRY(launch_site(AX{P.scal, P.red, nq, x, P.ps, nx, P.r, o.qa(), o.rcopy(), M},
                           [&](const AX& one, const AX* many, int count) {
                               if (many) hipLaunchKernelGGL((update_xr_kernel<T, T, true>), dim3(1024, count), dim3(RT), 0, st, one,
                                                  many);
        else hipLaunchKernelGGL((update_xr_kernel<T, T, false>), dim3(1024, count), dim3(RT), 0, st, one,
                                                  many);
                               return hipGetLastError();
                           }));
    GS_HIP_TRY(apply_TH_norm<T>(P, o.ra(), o.sa(), st, ns));
    using AP = UpdatePArgs<T, T>;
    return launch_site(AP{P.scal, P.red, ns, hist, hist_len, P.ps, o.sa(), o.pcopy(), nx, (const cx<double>*)x,
                          o.xbest()},
                       [&](const AP& one, const AP* many, int count) {
                           if (many) hipLaunchKernelGGL((update_p_kernel<T, T, true>), dim3(256, count), dim3(RT), 0, st,
                                                        one, many);
                           else hipLaunchKernelGGL((update_p_kernel<T, T, false>), dim3(256, count), dim3(RT), 0, st,
                                                   one, many);
                           return hipGetLastError();
                       });
}

// r = b - A x with applies of type T (x FP64 on device)
template <class T>
hipError_t compute_residual(const Plan& P, const cx<double>* x, hipStream_t st) {
    Ops<T> o{P};
    const int64_t nx = P.dim == 2 ? (int64_t)P.N * P.N : P.N;
    const cx<T>* xin;
    if constexpr (std::is_same<T, float>::value) {
        hipLaunchKernelGGL((convert_kernel<float>), dim3(nb256(nx)), dim3(256), 0, st, x, P.p32, nx);
        xin = P.p32;
    } else {
        xin = x;
    }
    GS_HIP_TRY(launch_apply_T<T>(P, xin, o.qa(), AFLAGS, st));
    hipLaunchKernelGGL((residual_kernel<T, T>), dim3(nb256(P.M)), dim3(256), 0, st, P.b, o.qa(), P.M, P.r,
                       o.rcopy());
    return hipGetLastError();
}

// run iterations until done or budget spent; returns iterations used (device count read back)
template <class T>
hipError_t cgls_run(const Plan& P, cx<double>* x, hipStream_t st, int budget, int check_every, double* hist,
                    int hist_len, bool& done, bool& broke) {
    done = false;
    broke = false;
    int it = 0, n = std::min(check_every, budget);
    double g_last = -1.0;
    int it_last = 0;
    while (it < budget) {
        for (int k = 0; k < n; ++k) GS_HIP_TRY(cgls_iteration<T>(P, x, st, hist, hist_len));
        it += n;
        GS_HIP_TRY(hipMemcpyAsync(P.host_scal, P.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
        GS_HIP_TRY(hipStreamSynchronize(st));
        if (P.host_scal[S_BREAK] != 0.0) {
            broke = true;
            return hipSuccess;
        }
        if (P.host_scal[S_DONE] != 0.0) {
            done = true;
            return hipSuccess;
        }
        // Iterations queued after the stop test passes run the applies for
        // nothing, so the next batch is cut to the iteration count the
        // observed rate of decrease of gamma predicts for reaching the
        // tolerance (the iterates do not depend on where the checks fall).
        int next = check_every;
        const double g = P.host_scal[S_GAMMA], ref = P.host_scal[S_REF];
        const double target = P.host_scal[S_TOL2] * ref * ref;
        const int it_dev = (int)P.host_scal[S_ITER];
        if (g_last > 0.0 && g < g_last && it_dev > it_last && target > 0.0) {
            const double rate = std::log(g / g_last) / (it_dev - it_last);
            const double need = std::log(target / g) / rate;
            if (std::isfinite(need) && need < next) next = std::max(1, (int)std::ceil(need));
        }
        g_last = g;
        it_last = it_dev;
        n = std::min(next, budget - it);
    }
    return hipSuccess;
}

// b, reference ||A^H b||, initial residual (x0 = 0 or warm start), s, gamma, p
template <class T>
int solve_setup(const Plan& P, const cx<double>* y, cx<double>* x, const gs_solve_opts& opt, hipStream_t st,
                int* warm_used) {
    const int64_t nx = P.dim == 2 ? (int64_t)P.N * P.N : P.N;
    const int64_t M = P.M;
    Ops<T> o{P};
    auto hipok = [&](hipError_t e) { return e == hipSuccess; };
    double* hist = opt.history ? P.hist : nullptr;
    const int hist_len = std::min(P.hist_len, opt.history_len);
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st, P.scal, (int)S_TOL2, opt.rel_tol * opt.rel_tol);
    // FP32 applies (mixed form) stop when the normal residual has grown 100x
    // over its smallest value; the FP64 refinement then restarts them
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st, P.scal, (int)S_GROW,
                       std::is_same<T, float>::value ? 1e4 : 0.0);
    hipLaunchKernelGGL((init_b_kernel<T>), dim3(nb256(M)), dim3(256), 0, st, y, P.perm, P.smu64, M, P.b, P.r,
                       o.rcopy());
    if (!hipok(hipGetLastError())) return GS_ERR_HIP;
    // reference ||A^H b|| (in apply precision T)
    if (!hipok(launch_apply_TH<T>(P, o.ra(), o.sa(), AFLAGS, st))) return GS_ERR_HIP;
    if (!hipok(launch_norm2<T>(o.sa(), nx, P.red, st))) return GS_ERR_HIP;
    hipLaunchKernelGGL(start_scalars_kernel, dim3(1), dim3(RT), 0, st, P.scal, P.red, RB, 1, nullptr, 0);
    bool warm = opt.warm_start != 0;
    if (warm) {
        if (!hipok(compute_residual<T>(P, x, st))) return GS_ERR_HIP;
    } else {
        hipLaunchKernelGGL((zero_kernel<double>), dim3(nb256(nx)), dim3(256), 0, st, x, nx);
    }
    if (!hipok(cgls_start<T>(P, x, st, 0, hist, hist_len))) return GS_ERR_HIP;
    if (warm && opt.warm_start == 2) {
        // guarded start: keep x0 only if ||A^H(b - A x0)|| < ||A^H b|| (zero start's value)
        if (!hipok(hipMemcpyAsync(P.host_scal, P.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st)) ||
            !hipok(hipStreamSynchronize(st)))
            return GS_ERR_HIP;
        const double g = P.host_scal[S_GAMMA], ref = P.host_scal[S_REF];
        if (!(g < ref * ref)) {
            warm = false;
            hipLaunchKernelGGL((zero_kernel<double>), dim3(nb256(nx)), dim3(256), 0, st, x, nx);
            hipLaunchKernelGGL((init_b_kernel<T>), dim3(nb256(M)), dim3(256), 0, st, y, P.perm, P.smu64, M, P.b,
                               P.r, o.rcopy());
            if (!hipok(cgls_start<T>(P, x, st, 0, hist, hist_len))) return GS_ERR_HIP;
        }
    }
    if (warm_used) *warm_used = warm ? 1 : 0;
    return GS_OK;
}

// after the recurrence stopped: the FP64 refinement (mixed form), history and info
template <class T>
int solve_finish(const Plan& P, cx<double>* x, const gs_solve_opts& opt, gs_solve_info& info, hipStream_t st,
                 bool done, bool broke) {
    const int64_t nx = P.dim == 2 ? (int64_t)P.N * P.N : P.N;
    const int64_t M = P.M;
    Ops<T> o{P};
    auto hipok = [&](hipError_t e) { return e == hipSuccess; };
    const int hist_len = std::min(P.hist_len, opt.history_len);
    int used = (int)P.host_scal[S_ITER], restarts = 0;
    double rel = P.host_scal[S_REF] > 0 ? std::sqrt(P.host_scal[S_GAMMA]) / P.host_scal[S_REF] : 0.0;
    double rel64 = -1;
    const bool refine = opt.refine_fp64 && std::is_same<T, float>::value && P.d64.present;
    // A stall (the reduced-precision recurrence passed its accuracy floor) ends
    // the run without a breakdown: x goes back to the run's best iterate and
    // the status follows the residual.
    auto settle_stall = [&]() {
        if (P.host_scal[S_STALL] == 0.0 || !o.xbest()) return;
        hipLaunchKernelGGL(copy_kernel, dim3(nb256(nx)), dim3(256), 0, st, (const cx<double>*)o.xbest(), x, nx);
        broke = false;
        rel = P.host_scal[S_REF] > 0 ? std::sqrt(P.host_scal[S_GMIN]) / P.host_scal[S_REF] : 0.0;
    };
    settle_stall();
    // mixed form: a stop of the FP32 recurrence (stall or breakdown) is not
    // final; the FP64 residual decides, and restarts resume from x
    if (refine) {
        // FP64 reference ||A^H b|| and recomputed FP64 residual
        if (!hipok(launch_apply_TH<double>(P, P.b, P.ss, AFLAGS, st))) return GS_ERR_HIP;
        if (!hipok(launch_norm2<double>(P.ss, nx, P.red, st))) return GS_ERR_HIP;
        hipLaunchKernelGGL(set_ref64_kernel, dim3(1), dim3(RT), 0, st, P.scal, P.red);
        for (;;) {
            if (!hipok(compute_residual<double>(P, x, st))) return GS_ERR_HIP;
            if (!hipok(launch_apply_TH<double>(P, P.r, P.ss, AFLAGS, st))) return GS_ERR_HIP;
            if (!hipok(launch_norm2<double>(P.ss, nx, P.red, st))) return GS_ERR_HIP;
            std::vector<double> red(RB);
            if (!hipok(hipMemcpyAsync(red.data(), P.red, RB * sizeof(double), hipMemcpyDeviceToHost, st)))
                return GS_ERR_HIP;
            if (!hipok(hipMemcpyAsync(P.host_scal, P.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st)))
                return GS_ERR_HIP;
            if (!hipok(hipStreamSynchronize(st))) return GS_ERR_HIP;
            double g = 0;
            for (double v : red) g += v;
            const double ref64 = P.host_scal[S_REF64];
            rel64 = ref64 > 0 ? std::sqrt(g) / ref64 : 0.0;
            if (rel64 <= opt.rel_tol || restarts >= opt.max_restarts || used >= opt.max_iter) break;
            ++restarts;
            // restart the FP32 recurrence from x with the FP64 residual
            hipLaunchKernelGGL((convert_kernel<T>), dim3(nb256(M)), dim3(256), 0, st, P.r, o.ra(), M);
            if (!hipok(cgls_start<T>(P, x, st, 0, nullptr, 0))) return GS_ERR_HIP;
            if (!hipok(cgls_run<T>(P, x, st, opt.max_iter - used, std::max(1, opt.check_every), nullptr, 0, done,
                                   broke)))
                return GS_ERR_HIP;
            used += (int)P.host_scal[S_ITER];
            rel = P.host_scal[S_REF] > 0 ? std::sqrt(P.host_scal[S_GAMMA]) / P.host_scal[S_REF] : 0.0;
            settle_stall();
        }
        done = rel64 <= opt.rel_tol;
        broke = !std::isfinite(rel64);
    }
    if (opt.history && hist_len > 0) {
        const int n = std::min(hist_len, used + 1);
        if (!hipok(hipMemcpyAsync(opt.history, P.hist, n * sizeof(double), hipMemcpyDeviceToHost, st)))
            return GS_ERR_HIP;
    }
    if (!hipok(hipStreamSynchronize(st))) return GS_ERR_HIP;
    info.iterations = used;
    info.restarts = restarts;
    info.rel_residual = rel;
    info.rel_residual_fp64 = rel64;
    info.status = broke ? GS_ERR_BREAKDOWN : (done ? GS_OK : GS_NOT_CONVERGED);
    return info.status;
}

template <class T>
int solve_impl(const Plan& P, const cx<double>* y, cx<double>* x, const gs_solve_opts& opt, gs_solve_info& info,
               hipStream_t st) {
    double* hist = opt.history ? P.hist : nullptr;
    const int hist_len = std::min(P.hist_len, opt.history_len);
    int warm_used = 0;
    int rc = solve_setup<T>(P, y, x, opt, st, &warm_used);
    if (rc != GS_OK) return rc;
    info.warm_start_used = warm_used;
    bool done = false, broke = false;
    if (cgls_run<T>(P, x, st, opt.max_iter, std::max(1, opt.check_every), hist, hist_len, done, broke) != hipSuccess)
        return GS_ERR_HIP;
    return solve_finish<T>(P, x, opt, info, st, done, broke);
}

// ------------------------------------------------------------------ batched solve
//
// Many independent problems (each with its own plan) advance together.
// Problems whose plans share one geometry -- the 2D tile path, the apply
// precision, N, the grid side and the number of boundary functions -- form a
// class.  A class runs each kernel of the CGLS iteration as ONE launch for all
// of its active problems (gridDim.y = problems): the launch code of the
// iteration runs once per problem in RECORD mode, which collects every launch
// site's argument struct, and the structs are uploaded as one device array per
// site (see LaunchCtx).  A round advances every active problem by one
// iteration; the rounds of a class are captured as HIP graphs (one iteration,
// and `ipg` iterations back to back) and replayed on the class's stream.
// Plans outside the tile path (1D, grids narrower than a tile) form classes of
// one problem with plain launches.  Every `check_every` rounds one host
// synchronization reads all stop flags.  Problems that are done leave their
// class: when at most 3/4 of the problems a class's graphs cover are still
// active, its argument arrays are compacted and its graphs recaptured.  The
// update kernels test the device stop flag, so the rounds a finished problem
// still takes part in change nothing.  Per problem, the kernels, their
// arithmetic and their order are those of gs_solve, so every result equals
// the lone solve's bit for bit.
//
// Tuner (n_streams = 0): the number of streams the classes are spread over
// (1, 2, 4 or 8; classes placed heaviest first) is picked from short timed
// trial rounds of the real iteration, which count as iterations.  Tile side
// and stage size are not tuned: they set the summation order inside a tile,
// and a batched problem must reproduce its lone solve and repeated runs
// must agree bit for bit.

struct BatchItem {
    const Plan* P;
    cx<double>* x;
    bool fp32;
    bool active = true, done = false, broke = false;
    int warm_used = 0;
    int cls = -1;
};

struct BatchClass {
    std::vector<int> members;                      // problem indices, class order
    std::vector<int> captured;                     // positions in members covered by the graphs
    bool batched = false;                          // kernel-batched launches
    bool fp32 = false;
    int stream = 0;
    double weight = 0;                             // sum of M + 4 ng^2 over members
    std::vector<size_t> sizes;                     // per launch site: struct size
    std::vector<std::vector<unsigned char>> rec;   // per site: the structs of all members
    std::vector<void*> dev;                        // per site: device array for `captured`
    hipGraph_t graph[2] = {nullptr, nullptr};      // one iteration; ipg iterations
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

static bool batchable(const Plan& P) { return P.dim == 2 && P.ts == TILE; }

template <class T>
static hipError_t iterate_as(const Plan& P, cx<double>* x, hipStream_t st) {
    return cgls_iteration<T>(P, x, st, nullptr, 0);
}

static hipError_t iterate(const BatchItem& it, hipStream_t st) {
    return it.fp32 ? iterate_as<float>(*it.P, it.x, st) : iterate_as<double>(*it.P, it.x, st);
}

// every launch site's argument structs of the class, member by member
static hipError_t record_class(BatchClass& c, const std::vector<BatchItem>& items, hipStream_t st) {
    c.rec.clear();
    c.sizes.clear();
    for (size_t k = 0; k < c.members.size(); ++k) {
        std::vector<std::vector<unsigned char>> one;
        LaunchCtx ctx;
        ctx.mode = LaunchCtx::RECORD;
        ctx.rec = &one;
        const bool prof = g_prof_enabled;   // nothing is launched: no timing records
        g_prof_enabled = false;
        g_launch = &ctx;
        const hipError_t e = iterate(items[c.members[k]], st);
        g_launch = nullptr;
        g_prof_enabled = prof;
        GS_HIP_TRY(e);
        if (k == 0) {
            c.rec.resize(one.size());
            for (auto& v : one) c.sizes.push_back(v.size());
        }
        if (one.size() != c.sizes.size()) return hipErrorInvalidValue;
        for (size_t i = 0; i < one.size(); ++i) {
            if (one[i].size() != c.sizes[i]) return hipErrorInvalidValue;
            c.rec[i].insert(c.rec[i].end(), one[i].begin(), one[i].end());
        }
    }
    return hipSuccess;
}

static void drop_graphs(BatchClass& c) {
    for (int w = 0; w < 2; ++w) {
        if (c.exec[w]) (void)hipGraphExecDestroy(c.exec[w]);
        if (c.graph[w]) (void)hipGraphDestroy(c.graph[w]);
        c.exec[w] = nullptr;
        c.graph[w] = nullptr;
    }
}

static void drop_arrays(BatchClass& c) {
    for (void* d : c.dev) (void)hipFree(d);
    c.dev.clear();
}

// argument arrays of the captured members (caller has synchronized the class's stream)
static hipError_t upload_class(BatchClass& c) {
    drop_arrays(c);
    for (size_t i = 0; i < c.sizes.size(); ++i) {
        const size_t sz = c.sizes[i];
        std::vector<unsigned char> buf(sz * c.captured.size());
        for (size_t k = 0; k < c.captured.size(); ++k)
            std::copy_n(&c.rec[i][sz * c.captured[k]], sz, &buf[sz * k]);
        void* d = nullptr;
        GS_HIP_TRY(hipMalloc(&d, buf.size()));
        c.dev.push_back(d);
        GS_HIP_TRY(hipMemcpy(d, buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
    return hipSuccess;
}

static hipError_t capture_class(BatchClass& c, const std::vector<BatchItem>& items, int which, int iters,
                                hipStream_t cs) {
    const BatchItem& rep = items[c.members[c.captured[0]]];
    LaunchCtx ctx;
    ctx.mode = LaunchCtx::BATCH;
    ctx.dev = c.dev.data();
    ctx.sizes = c.sizes.data();
    ctx.nsites = (int)c.sizes.size();
    ctx.count = (int)c.captured.size();
    // per-kernel timing events are host-side records: none inside a graph
    const bool prof = g_prof_enabled;
    g_prof_enabled = false;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int k = 0; k < iters && e == hipSuccess; ++k) {
        if (c.batched) {
            ctx.site = 0;
            g_launch = &ctx;
        }
        e = iterate(rep, cs);
        g_launch = nullptr;
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    g_prof_enabled = prof;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    GS_HIP_TRY(e2);
    c.graph[which] = g;
    return hipGraphInstantiate(&c.exec[which], g, nullptr, nullptr, 0);
}

static hipError_t build_class_graphs(BatchClass& c, const std::vector<BatchItem>& items, int ipg, hipStream_t cs) {
    drop_graphs(c);
    if (c.captured.empty()) return hipSuccess;
    if (c.batched) GS_HIP_TRY(upload_class(c));
    GS_HIP_TRY(capture_class(c, items, 0, 1, cs));
    if (ipg > 1) GS_HIP_TRY(capture_class(c, items, 1, ipg, cs));
    return hipSuccess;
}

static void assign_streams(std::vector<BatchClass>& cls, int ns) {
    std::vector<int> order(cls.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls[a].weight > cls[b].weight; });
    std::vector<double> load(ns, 0.0);
    for (int i : order) {
        const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        cls[i].stream = s;
        load[s] += cls[i].weight;
    }
}

}  // namespace gs

extern "C" int gs_solve_batch(const gs_plan_t* const* plans, int count, const void* const* y, void* const* x,
                              const gs_solve_opts* opts, gs_solve_info* infos, int n_streams, void* stream) {
    using namespace gs;
    if (!plans || count < 1 || !y || !x || !opts || !infos) return GS_ERR_INVALID_ARG;
    if (!(opts->rel_tol >= 0) || opts->max_iter < 1 || opts->max_restarts < 0) return GS_ERR_INVALID_ARG;
    if (opts->warm_start < 0 || opts->warm_start > 2) return GS_ERR_INVALID_ARG;
    if (opts->history) return GS_ERR_INVALID_ARG;  // one host history buffer cannot serve several problems
    if (n_streams < 0 || n_streams > 64) return GS_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !y[i] || !x[i]) return GS_ERR_INVALID_ARG;
        // each problem owns its plan's work vectors and its own solution
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i] || x[j] == x[i]) return GS_ERR_INVALID_ARG;
    }
    hipStream_t user = (hipStream_t)stream;
    std::vector<BatchItem> items(count);
    std::vector<BatchClass> cls;
    std::vector<hipStream_t> streams;
    hipEvent_t ev0 = nullptr;
    auto cleanup = [&]() {
        for (auto s : streams) (void)hipStreamSynchronize(s);
        for (auto& c : cls) {
            drop_graphs(c);
            drop_arrays(c);
        }
        if (ev0) (void)hipEventDestroy(ev0);
        for (auto s : streams) (void)hipStreamDestroy(s);
    };
    auto fail = [&](hipError_t) {
        cleanup();
        return GS_ERR_HIP;
    };
    // classes: one per geometry on the tile path, else one per problem
    for (int i = 0; i < count; ++i) {
        const Plan& P = plans[i]->impl;
        BatchItem& it = items[i];
        it.P = &P;
        it.x = (cx<double>*)x[i];
        it.fp32 = P.d32.present && P.precision != GS_F64;
        infos[i] = gs_solve_info{0, 0, GS_OK, -1.0, -1.0, 0, -1, 0};
        int c = -1;
        if (batchable(P))
            for (size_t k = 0; k < cls.size() && c < 0; ++k) {
                const Plan& Q = *items[cls[k].members[0]].P;
                if (cls[k].batched && cls[k].fp32 == it.fp32 && Q.N == P.N && Q.ng == P.ng && Q.nb == P.nb &&
                    Q.cr1 == P.cr1)
                    c = (int)k;
            }
        if (c < 0) {
            cls.emplace_back();
            c = (int)cls.size() - 1;
            cls[c].batched = batchable(P);
            cls[c].fp32 = it.fp32;
        }
        it.cls = c;
        cls[c].members.push_back(i);
        cls[c].weight += (double)P.M + 4.0 * P.ng * P.ng;
    }
    const int ncls = (int)cls.size();
    // at most 8 internal streams: more than the device's hardware queues only take turns
    const int ns_max = std::min({n_streams > 0 ? n_streams : 8, 8, ncls});
    for (int s = 0; s < ns_max; ++s) {
        hipStream_t h;
        if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) return fail(hipErrorUnknown);
        streams.push_back(h);
    }
    if (hipEventCreateWithFlags(&ev0, hipEventDisableTiming) != hipSuccess) return fail(hipErrorUnknown);
    if (hipEventRecord(ev0, user) != hipSuccess) return fail(hipErrorUnknown);
    for (auto s : streams)
        if (hipStreamWaitEvent(s, ev0, 0) != hipSuccess) return fail(hipErrorUnknown);
    assign_streams(cls, ns_max);
    // set-up of every problem (plain launches on its class's stream)
    for (auto& it : items) {
        hipStream_t s = streams[cls[it.cls].stream];
        const cx<double>* yi = (const cx<double>*)y[&it - items.data()];
        int wu = 0;
        const int rc = it.fp32 ? solve_setup<float>(*it.P, yi, it.x, *opts, s, &wu)
                               : solve_setup<double>(*it.P, yi, it.x, *opts, s, &wu);
        it.warm_used = wu;
        if (rc != GS_OK) {
            cleanup();
            return rc;
        }
    }
    const int check_every = std::max(1, opts->check_every);
    // iterations per graph launch: up to 16 captured back to back, the rest of
    // a check interval from the one-iteration graph
    const int ipg = std::min(check_every, 16);
    for (auto& c : cls) {
        hipStream_t s = streams[c.stream];
        for (size_t k = 0; k < c.members.size(); ++k) c.captured.push_back((int)k);
        if (c.batched && record_class(c, items, s) != hipSuccess) return fail(hipErrorUnknown);
        if (build_class_graphs(c, items, ipg, s) != hipSuccess) return fail(hipErrorUnknown);
    }
    int ns = ns_max;
    int rounds = 0;
    auto class_active = [&](const BatchClass& c) {
        for (int k : c.captured)
            if (items[c.members[k]].active) return true;
        return false;
    };
    // n rounds: every active problem advances by n iterations
    auto run_rounds = [&](int n) -> hipError_t {
        const int full = ipg > 1 ? n / ipg : 0, rest = n - full * ipg;
        for (int r = 0; r < full; ++r)
            for (auto& c : cls)
                if (class_active(c)) GS_HIP_TRY(hipGraphLaunch(c.exec[1], streams[c.stream]));
        for (int r = 0; r < rest; ++r)
            for (auto& c : cls)
                if (class_active(c)) GS_HIP_TRY(hipGraphLaunch(c.exec[0], streams[c.stream]));
        return hipSuccess;
    };
    auto check = [&]() -> hipError_t {
        for (auto& it : items)
            if (it.active)
                GS_HIP_TRY(hipMemcpyAsync(it.P->host_scal, it.P->scal, S_NSCAL * sizeof(double),
                                          hipMemcpyDeviceToHost, streams[cls[it.cls].stream]));
        for (int s = 0; s < ns_max; ++s) GS_HIP_TRY(hipStreamSynchronize(streams[s]));
        for (auto& it : items) {
            if (!it.active) continue;
            const double* h = it.P->host_scal;
            if (h[S_BREAK] != 0.0) {
                it.broke = true;
                it.active = false;
            } else if (h[S_DONE] != 0.0) {
                it.done = true;
                it.active = false;
            } else if ((int)h[S_ITER] >= opts->max_iter) {
                it.active = false;
            }
        }
        // classes whose graphs cover many finished problems: compact and recapture
        for (auto& c : cls) {
            if (!c.batched || c.captured.empty()) continue;
            std::vector<int> keep;
            for (int k : c.captured)
                if (items[c.members[k]].active) keep.push_back(k);
            if (keep.size() == c.captured.size() || 4 * keep.size() > 3 * c.captured.size()) continue;
            c.captured = keep;
            GS_HIP_TRY(build_class_graphs(c, items, ipg, streams[c.stream]));
        }
        return hipSuccess;
    };
    auto any_active = [&]() {
        for (auto& it : items)
            if (it.active) return true;
        return false;
    };
    if (n_streams == 0 && ns_max > 1) {
        // trial: candidate stream counts, a few real rounds each
        const int trial = std::min(std::max(3, ipg), opts->max_iter);
        double best = 1e300;
        int best_ns = ns_max;
        for (int cand = 1; cand <= ns_max && rounds + trial <= opts->max_iter && any_active(); cand *= 2) {
            ns = cand;
            for (int s = 0; s < ns_max; ++s)
                if (hipStreamSynchronize(streams[s]) != hipSuccess) return fail(hipErrorUnknown);
            assign_streams(cls, ns);
            const auto t0 = std::chrono::steady_clock::now();
            if (run_rounds(trial) != hipSuccess) return fail(hipErrorUnknown);
            for (int s = 0; s < ns; ++s)
                if (hipStreamSynchronize(streams[s]) != hipSuccess) return fail(hipErrorUnknown);
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            rounds += trial;
            if (dt < best) {
                best = dt;
                best_ns = cand;
            }
            if (check() != hipSuccess) return fail(hipErrorUnknown);
        }
        ns = best_ns;
        assign_streams(cls, ns);  // every stream is idle after the last check
    }
    while (any_active() && rounds < opts->max_iter) {
        const int n = std::min(check_every, opts->max_iter - rounds);
        if (run_rounds(n) != hipSuccess) return fail(hipErrorUnknown);
        rounds += n;
        if (check() != hipSuccess) return fail(hipErrorUnknown);
    }
    for (int s = 0; s < ns_max; ++s)
        if (hipStreamSynchronize(streams[s]) != hipSuccess) return fail(hipErrorUnknown);
    // refinement (mixed form) and results, one problem after the other on the caller's stream
    int worst = GS_OK;
    for (int i = 0; i < count; ++i) {
        BatchItem& it = items[i];
        if (hipMemcpy(it.P->host_scal, it.P->scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(hipErrorUnknown);
        const int r = it.fp32 ? solve_finish<float>(*it.P, it.x, *opts, infos[i], user, it.done, it.broke)
                              : solve_finish<double>(*it.P, it.x, *opts, infos[i], user, it.done, it.broke);
        infos[i].warm_start_used = it.warm_used;
        infos[i].batch_class = cls[it.cls].batched ? it.cls : -1;
        infos[i].batch_streams = ns;
        // every problem is finished and reported; the call returns the worst
        // status (an error before GS_NOT_CONVERGED before GS_OK)
        if (r < 0 && worst >= 0) worst = r;
        else if (r == GS_NOT_CONVERGED && worst == GS_OK) worst = r;
    }
    cleanup();
    return worst;
}

extern "C" int gs_solve(const gs_plan_t* plan, const void* y, void* x, const gs_solve_opts* opts,
                        gs_solve_info* info, void* stream);

extern "C" int gs_solve(const gs_plan_t* plan, const void* y, void* x, const gs_solve_opts* opts, gs_solve_info* info,
                        void* stream) {
    if (!plan || !y || !x || !opts) return GS_ERR_INVALID_ARG;
    if (!(opts->rel_tol >= 0) || opts->max_iter < 1 || opts->max_restarts < 0) return GS_ERR_INVALID_ARG;
    if (opts->warm_start < 0 || opts->warm_start > 2) return GS_ERR_INVALID_ARG;
    if (opts->history && opts->history_len < 1) return GS_ERR_INVALID_ARG;
    gs_solve_info local{};
    gs_solve_info& inf = info ? *info : local;
    inf = gs_solve_info{0, 0, GS_OK, -1.0, -1.0, 0, -1, 0};
    const gs::Plan& P = plan->impl;
    hipStream_t st = (hipStream_t)stream;
    if (P.d32.present && P.precision != GS_F64)
        return gs::solve_impl<float>(P, (const gs::cx<double>*)y, (gs::cx<double>*)x, *opts, inf, st);
    return gs::solve_impl<double>(P, (const gs::cx<double>*)y, (gs::cx<double>*)x, *opts, inf, st);
}
