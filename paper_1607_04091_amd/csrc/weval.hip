// Evaluation of a representation in V_J^int on dyadic grids (the paper's
// weval of the IntervalWavelets companion package, Sec. 6.2; Figs. 1-2):
//   f(x) = sum_n x_n s_n(x),  x = -1/2 + j 2^-R,  j = 0..2^R,
// with s_n the basis of Sec. 3.3: left boundary functions 2^{J/2}
// phi^L_n(2^J (x + 1/2)) for n < p, interior 2^{J/2} phi(2^J (x + 1/2) - n),
// right boundary functions 2^{J/2} phi^R_{N-1-n}(2^J (x - 1/2)) for n >= N - p
// (2D: the tensor product, f(x, y) = sum X[i][j] s_i(x) s_j(y)).
//
// Cascade algorithm: phi at the integers is the fixed point of the refinement
// equation phi(x) = 2 sum_k h_k phi(2x - k) on the integers (host); each
// device pass doubles the resolution with the same equation, up to
// r = R - J.  The boundary functions at resolution r are the linear
// combinations of restricted translates that define them (App. A.1):
// phi^L_k(t) = sum_n c_{n,k} phi(t - n) for t >= 0, and phi^R_k(t) =
// phi^{bL}_k(-t) with the reflected filter, whose scaling function is
// phi(1 - t).  All arithmetic is FP64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "host_math.hpp"

namespace gs {

namespace {

constexpr int WE_THREADS = 256;

// one doubling step: out[j] = phi(j / 2^r) for j in [lo 2^r, hi 2^r], from
// in[j'] = phi(j' / 2^(r-1)), j' in [lo 2^(r-1), hi 2^(r-1)]
__global__ void cascade_kernel(const double* __restrict__ in, double* __restrict__ out, const double* __restrict__ h,
                               int p, int r) {
    const int lo = -p + 1, hi = p;
    const int64_t n_out = (int64_t)(hi - lo) * ((int64_t)1 << r) + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int64_t j = i + (int64_t)lo * ((int64_t)1 << r);
    const int64_t half = (int64_t)1 << (r - 1), in_lo = (int64_t)lo * half, n_in = (int64_t)(hi - lo) * half + 1;
    double s = 0.0;
    for (int k = lo; k <= hi; ++k) {
        const int64_t src = j - (int64_t)k * half - in_lo;
        if (src >= 0 && src < n_in) s += 2.0 * h[k - lo] * in[src];
    }
    out[i] = s;
}

struct Tables {
    const double* phi;    // phi(j / 2^r), j from lo 2^r
    const double* bl;     // [p][B] phi^L_k(j / 2^r), j = 0..B-1
    const double* br;     // [p][B] phi^R_k(-j / 2^r), j = 0..B-1
    int p, nb, r, lo;
    int64_t nphi, B;
    __device__ double phi_at(int64_t num) const {   // phi(num / 2^r)
        const int64_t i = num - (int64_t)lo * ((int64_t)1 << r);
        return (i >= 0 && i < nphi) ? phi[i] : 0.0;
    }
};

// boundary functions at resolution r from the restricted translates
__global__ void boundary_tables_kernel(Tables t, const double* __restrict__ cl, const double* __restrict__ cr,
                                       double* __restrict__ bl, double* __restrict__ br) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)t.p * t.B) return;
    const int k = (int)(i / t.B);
    const int64_t j = i - (int64_t)k * t.B;
    const int64_t one = (int64_t)1 << t.r;
    double sl = 0.0, sr = 0.0;
    for (int n = -t.p + 1; n <= t.p - 1; ++n) {
        const double al = cl[(n + t.p - 1) * t.p + k], ar = cr[(n + t.p - 1) * t.p + k];
        sl += al * t.phi_at(j - n * one);              // phi^L_k(j / 2^r), j / 2^r >= 0
        sr += ar * t.phi_at(one - j + n * one);        // phi^R_k(-j / 2^r) = sum a phi(1 - j / 2^r + n)
    }
    bl[i] = sl;
    br[i] = sr;
}

// value of basis function n of the scale-J basis at t = 2^J (x + 1/2) = num / 2^r
__device__ inline double basis_at(const Tables& tb, int N, int n, int64_t num) {
    const int64_t one = (int64_t)1 << tb.r;
    if (n < tb.nb) return (num >= 0 && num < tb.B) ? tb.bl[(int64_t)n * tb.B + num] : 0.0;
    if (n >= N - tb.nb) {
        const int k = N - 1 - n;
        const int64_t m = (int64_t)N * one - num;        // -(t - N) in units of 2^-r
        return (m >= 0 && m < tb.B) ? tb.br[(int64_t)k * tb.B + m] : 0.0;
    }
    return tb.phi_at(num - (int64_t)n * one);
}

// the basis functions that can be nonzero at t = num / 2^r: interior n with
// t - n in (-p+1, p), and the boundary functions near either end
__device__ inline int basis_list(const Tables& tb, int N, int64_t num, int* idx, double* val) {
    const int64_t one = (int64_t)1 << tb.r;
    const int64_t tf = num >> tb.r;   // floor(t)
    int cnt = 0;
    for (int64_t n = tf - tb.p + 1; n <= tf + tb.p - 1; ++n) {
        if (n < tb.nb || n >= N - tb.nb) continue;
        const double v = tb.phi_at(num - n * one);
        if (v != 0.0) { idx[cnt] = (int)n; val[cnt] = v; ++cnt; }
    }
    for (int k = 0; k < tb.nb; ++k) {
        double v = basis_at(tb, N, k, num);
        if (v != 0.0) { idx[cnt] = k; val[cnt] = v; ++cnt; }
        v = basis_at(tb, N, N - 1 - k, num);
        if (v != 0.0) { idx[cnt] = N - 1 - k; val[cnt] = v; ++cnt; }
    }
    return cnt;
}

constexpr int MAXB = 48;   // >= 2p - 1 interior + 2p boundary functions for p <= 8

__global__ void weval1d_kernel(Tables tb, int N, int J, int R, const cx<double>* __restrict__ c,
                               cx<double>* __restrict__ f) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > ((int64_t)1 << R)) return;
    // t = 2^J (x + 1/2) = j 2^(J - R) = j / 2^r
    int idx[MAXB];
    double val[MAXB];
    const int cnt = basis_list(tb, N, j, idx, val);
    const double sc = ldexp(1.0, 0) * sqrt(ldexp(1.0, J));
    cx<double> s = czero<double>();
    for (int i = 0; i < cnt; ++i) s = cfma(s, c[idx[i]], val[i]);
    f[j] = cscale(s, sc);
}

__global__ void weval2d_kernel(Tables tb, int N, int J, int R, const cx<double>* __restrict__ X,
                               cx<double>* __restrict__ f) {
    const int64_t side = ((int64_t)1 << R) + 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= side * side) return;
    const int64_t jx = e / side, jy = e - jx * side;
    int ix[MAXB], iy[MAXB];
    double vx[MAXB], vy[MAXB];
    const int nx = basis_list(tb, N, jx, ix, vx);
    const int ny = basis_list(tb, N, jy, iy, vy);
    cx<double> s = czero<double>();
    for (int a = 0; a < nx; ++a) {
        const cx<double>* row = X + (size_t)ix[a] * N;
        cx<double> t = czero<double>();
        for (int b = 0; b < ny; ++b) t = cfma(t, row[iy[b]], vy[b]);
        s = cfma(s, t, vx[a]);
    }
    f[e] = cscale(s, ldexp(1.0, J));   // 2^{J/2} per dimension
}

}  // namespace

}  // namespace gs

extern "C" int gs_weval(int dim, int J, int p, int R, const void* coef, void* out, void* stream) {
    using namespace gs;
    if (!coef || !out || (dim != 1 && dim != 2)) return GS_ERR_INVALID_ARG;
    if (p < 1 || p > 8 || J < 1 || J > (dim == 2 ? 11 : 20) || (1 << J) < 2 * p) return GS_ERR_UNSUPPORTED;
    if (R < J || R - J > 20 || R > (dim == 2 ? 13 : 26)) return GS_ERR_UNSUPPORTED;
    const BasisData* bd = nullptr;
    try {
        bd = &basis_data(p);
    } catch (...) {
        return GS_ERR_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    const int r = R - J, lo = -p + 1, hi = p, nb = p == 1 ? 0 : p;
    const int64_t nphi = (int64_t)(hi - lo) * ((int64_t)1 << r) + 1;
    // boundary tables cover t in [0, 2p - 1] (the support of every phi^L_k)
    const int64_t B = (int64_t)(2 * p - 1) * ((int64_t)1 << r) + 1;
    std::vector<void*> tmp;
    auto cleanup = [&](int rc) {
        (void)hipStreamSynchronize(s);
        for (void* v : tmp) (void)hipFree(v);
        return rc;
    };
    auto get = [&](double*& ptr, size_t n) -> hipError_t {
        void* v = nullptr;
        hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(double));
        if (e == hipSuccess) tmp.push_back(v);
        ptr = static_cast<double*>(v);
        return e;
    };
    double *a = nullptr, *b = nullptr, *h = nullptr, *bl = nullptr, *br = nullptr, *cl = nullptr, *cr = nullptr;
    if (get(a, nphi) || get(b, nphi) || get(h, 2 * p)) return cleanup(GS_ERR_NOMEM);
    if (hipMemcpyAsync(h, bd->taps.data(), 2 * p * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(a, bd->phi_int.data(), (hi - lo + 1) * sizeof(double), hipMemcpyHostToDevice, s))
        return cleanup(GS_ERR_HIP);
    for (int lev = 1; lev <= r; ++lev) {
        const int64_t n = (int64_t)(hi - lo) * ((int64_t)1 << lev) + 1;
        hipLaunchKernelGGL(cascade_kernel, dim3((int)((n + WE_THREADS - 1) / WE_THREADS)), dim3(WE_THREADS), 0, s, a, b,
                           h, p, lev);
        std::swap(a, b);
    }
    Tables tb{a, nullptr, nullptr, p, nb, r, lo, nphi, B};
    if (nb) {
        if (get(bl, (size_t)p * B) || get(br, (size_t)p * B) || get(cl, bd->left.coef.size()) ||
            get(cr, bd->right.coef.size()))
            return cleanup(GS_ERR_NOMEM);
        if (hipMemcpyAsync(cl, bd->left.coef.data(), bd->left.coef.size() * sizeof(double), hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(cr, bd->right.coef.data(), bd->right.coef.size() * sizeof(double), hipMemcpyHostToDevice,
                           s))
            return cleanup(GS_ERR_HIP);
        hipLaunchKernelGGL(boundary_tables_kernel, dim3((int)((p * B + WE_THREADS - 1) / WE_THREADS)), dim3(WE_THREADS),
                           0, s, tb, cl, cr, bl, br);
        tb.bl = bl;
        tb.br = br;
    }
    const int N = 1 << J;
    const int64_t side = ((int64_t)1 << R) + 1;
    if (dim == 1)
        hipLaunchKernelGGL(weval1d_kernel, dim3((int)((side + WE_THREADS - 1) / WE_THREADS)), dim3(WE_THREADS), 0, s, tb,
                           N, J, R, (const cx<double>*)coef, (cx<double>*)out);
    else
        hipLaunchKernelGGL(weval2d_kernel, dim3((int)((side * side + WE_THREADS - 1) / WE_THREADS)), dim3(WE_THREADS), 0,
                           s, tb, N, J, R, (const cx<double>*)coef, (cx<double>*)out);
    if (hipGetLastError() != hipSuccess) return cleanup(GS_ERR_HIP);
    return cleanup(GS_OK);
}
