// Host-side FP64/extended-precision math for plan construction:
// Daubechies taps, CDV boundary recursion data, per-point basis values and
// the Kaiser-Bessel window of the NFFT.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace gs {

using cd = std::complex<double>;

struct BoundaryEdge {
    std::vector<double> U;   // p x p row-major      (H / sqrt 2)
    std::vector<double> V;   // p x (2p-1) row-major (h / sqrt 2), columns m = p..3p-2
    std::vector<double> v0;  // v1(0)
    std::vector<double> coef;  // (2p-1) x p row-major: coefficient of the restricted
                               // translate phi(. - n), n = -p+1..p-1 (row), in phi^L_k (column)
};

struct BasisData {
    int p = 0;
    std::vector<double> taps;  // h_k, k = -p+1..p
    BoundaryEdge left, right;  // empty for p = 1
    std::vector<double> phi_int;  // phi at the integers -p+1..p (refinement eigenvector, sum 1)
};

// Cached per p (thread-safe).  Throws std::runtime_error if p unsupported.
const BasisData& basis_data(int p);

// Basis channel values at M points (see gs_eval_basis_1d): out[m*(2nb+1) + c].
void eval_basis_1d(int J, int p, int64_t M, const double* xi, int stride, cd* out, int nthreads);

// Kaiser-Bessel window phi(d) = I0(beta sqrt(1 - (2d/w)^2)) / I0(beta), |d| <= w/2,
// approximated per tap j by a degree-`deg` polynomial in x = 2t - 1 where
// t = frac(grid coordinate) and tap j sits at offset d = t + w/2 - 1 - j.
struct KBWindow {
    int w = 0, deg = 0;
    double beta = 0;
    std::vector<double> coef;  // w x (deg+1), ascending powers of x
    double eval_exact(double d) const;
    double ft(double f) const;  // continuous Fourier transform at frequency f (grid units)
};
KBWindow make_window(int w, int deg, double beta);

}  // namespace gs
