// Host math for plan construction (independent FP64 / x87-extended code).
//
// * Daubechies taps (App. A: m0(xi) = sum_k h_k e^{-2 pi i k xi}, m0(0) = 1):
//   spectral factorization of |m0|^2 = cos^{2p}(pi xi) P(sin^2 pi xi); the
//   p-1 roots of P are found by Durand-Kerner iteration, and for each the
//   zero of the minimum-phase factor outside the unit circle in
//   z = e^{-2 pi i xi} is kept.  Taps are indexed k = -p+1..p (Sec. 3.3).
// * CDV boundary functions (App. A.1): half-line Gram matrix from the
//   refinement identity, edge space of restricted polynomial sequences,
//   staircase orthonormalization through a Cholesky factor, then the
//   dilation filters H, h, the matrices U = H/sqrt2, V = h/sqrt2 and v1(0).
//   Right edge by reflection of the filter (h_k -> h_{1-k}).
// * Per-point values: phi-hat as the product of m0 over dyadic dilations
//   (App. A) and the boundary transforms by the dilation recursion
//   v1(xi) = U v1(xi/2) + V v2(xi/2) started from v1(0) (App. A.1).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <thread>

namespace gs {

using ld = long double;
using cld = std::complex<ld>;

namespace {

std::vector<ld> daubechies_taps(int p) {
    if (p == 1) return {0.5L, 0.5L};
    // P(y) = sum_{j<p} C(p-1+j, j) y^j
    std::vector<ld> P(p);
    for (int j = 0; j < p; ++j) {
        ld c = 1;
        for (int i = 1; i <= j; ++i) c = c * (p - 1 + i) / i;
        P[j] = c;
    }
    const int deg = p - 1;
    auto evalP = [&](cld y) {
        cld acc = 0;
        for (int j = deg; j >= 0; --j) acc = acc * y + P[j];
        return acc;
    };
    auto evaldP = [&](cld y) {
        cld acc = 0;
        for (int j = deg; j >= 1; --j) acc = acc * y + P[j] * (ld)j;
        return acc;
    };
    // Durand-Kerner on the monic polynomial P / P[deg]
    std::vector<cld> r(deg);
    const cld seed(0.4L, 0.9L);
    cld s = 1;
    for (int i = 0; i < deg; ++i) { s *= seed; r[i] = s; }
    for (int it = 0; it < 2000; ++it) {
        ld delta = 0;
        for (int i = 0; i < deg; ++i) {
            cld den = P[deg];
            for (int k = 0; k < deg; ++k)
                if (k != i) den *= (r[i] - r[k]);
            cld step = evalP(r[i]) / den;
            r[i] -= step;
            delta = std::max(delta, std::abs(step));
        }
        if (delta < 1e-30L) break;
    }
    for (int i = 0; i < deg; ++i)
        for (int it = 0; it < 4; ++it) r[i] -= evalP(r[i]) / evaldP(r[i]);
    // polynomial in z, ascending: ((1+z)/2)^p * prod (z - z_r)
    std::vector<cld> poly{1};
    auto mul = [&](cld a0, cld a1) {
        std::vector<cld> out(poly.size() + 1, 0);
        for (size_t i = 0; i < poly.size(); ++i) {
            out[i] += poly[i] * a0;
            out[i + 1] += poly[i] * a1;
        }
        poly.swap(out);
    };
    for (int i = 0; i < p; ++i) mul(0.5L, 0.5L);
    for (int i = 0; i < deg; ++i) {
        cld b = (ld)1 - (ld)2 * r[i];
        cld sq = std::sqrt(b * b - (ld)1);
        cld z = (std::abs(b + sq) > 1) ? b + sq : b - sq;
        mul(-z, 1);
    }
    cld tot = 0;
    for (auto& c : poly) tot += c;
    std::vector<ld> h(poly.size());
    for (size_t i = 0; i < poly.size(); ++i) h[i] = std::real(poly[i] / tot);
    return h;
}

// Gaussian elimination with partial pivoting, A (n x n row-major), b overwritten.
void solve_dense(std::vector<ld>& A, std::vector<ld>& b, int n) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0) throw std::runtime_error("singular system in boundary construction");
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            ld f = A[r * n + c] / A[c * n + c];
            if (f == 0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        ld s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
}

// Left-edge construction for taps hk (index k + p - 1, k = -p+1..p).
BoundaryEdge edge_construction(const std::vector<ld>& hk, int p) {
    const int lo = -p + 1, hi = p - 2;  // unknown Gram range
    const int q = hi - lo + 1;           // 2p - 2
    // unknown index: symmetric pairs (a <= b)
    std::vector<int> pos(q * q, -1);
    int nu = 0;
    for (int a = 0; a < q; ++a)
        for (int b = a; b < q; ++b) pos[a * q + b] = pos[b * q + a] = nu++;
    auto known = [&](int n, int m, ld& v) {
        if (n >= p - 1 || m >= p - 1) { v = (n == m) ? 1 : 0; return true; }
        if (n <= -p || m <= -p) { v = 0; return true; }
        return false;
    };
    std::vector<ld> A(nu * nu, 0), rhs(nu, 0);
    for (int a = 0; a < q; ++a)
        for (int b = a; b < q; ++b) {
            const int row = pos[a * q + b];
            const int n = a + lo, m = b + lo;
            A[row * nu + row] += 1;
            for (int i = 0; i < 2 * p; ++i)
                for (int j = 0; j < 2 * p; ++j) {
                    const ld c = 2 * hk[i] * hk[j];
                    const int s = 2 * n + (i - p + 1), t = 2 * m + (j - p + 1);
                    ld v;
                    if (known(s, t, v)) rhs[row] += c * v;
                    else A[row * nu + pos[(s - lo) * q + (t - lo)]] -= c;
                }
        }
    if (nu > 0) solve_dense(A, rhs, nu);
    auto G = [&](int n, int m) -> ld {
        ld v;
        if (known(n, m, v)) return v;
        return rhs[pos[(n - lo) * q + (m - lo)]];
    };
    // edge space basis B ((2p-1) x p): column k = prod_{t=k+1}^{p-1} (n - t)
    const int nt = 2 * p - 1;  // translates n = -p+1..p-1
    std::vector<ld> B(nt * p);
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < p; ++k) {
            ld v = 1;
            for (int t = k + 1; t < p; ++t) v *= (ld)(i - p + 1 - t);
            B[i * p + k] = v;
        }
    // S = B^T G B, Cholesky S = L L^T, coefficients C = B L^{-T}
    std::vector<ld> GB(nt * p, 0), S(p * p, 0);
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < p; ++k) {
            ld s = 0;
            for (int j = 0; j < nt; ++j) s += G(i - p + 1, j - p + 1) * B[j * p + k];
            GB[i * p + k] = s;
        }
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            ld s = 0;
            for (int i = 0; i < nt; ++i) s += B[i * p + a] * GB[i * p + b];
            S[a * p + b] = s;
        }
    std::vector<ld> L(p * p, 0);
    for (int j = 0; j < p; ++j) {
        ld d = S[j * p + j];
        for (int k = 0; k < j; ++k) d -= L[j * p + k] * L[j * p + k];
        if (d <= 0) throw std::runtime_error("edge Gram matrix not positive definite");
        L[j * p + j] = std::sqrt(d);
        for (int i = j + 1; i < p; ++i) {
            ld s = S[i * p + j];
            for (int k = 0; k < j; ++k) s -= L[i * p + k] * L[j * p + k];
            L[i * p + j] = s / L[j * p + j];
        }
    }
    // Linv^T: solve L^T Y = I  -> Y upper triangular
    std::vector<ld> Y(p * p, 0);
    for (int c = 0; c < p; ++c) {
        for (int r = p - 1; r >= 0; --r) {
            ld s = (r == c) ? 1 : 0;
            for (int k = r + 1; k < p; ++k) s -= L[k * p + r] * Y[k * p + c];
            Y[r * p + c] = s / L[r * p + r];
        }
    }
    std::vector<ld> Cf(nt * p, 0);  // coefficient of translate n (row) in phi^L_k (col)
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < p; ++k) {
            ld s = 0;
            for (int l = 0; l <= k; ++l) s += B[i * p + l] * Y[l * p + k];
            Cf[i * p + k] = s;
        }
    for (int k = 0; k < p; ++k) {  // sign: coefficient of translate n = k positive
        if (Cf[(k + p - 1) * p + k] < 0)
            for (int i = 0; i < nt; ++i) Cf[i * p + k] = -Cf[i * p + k];
    }
    // refinement: phi(x-n) = sum_s 2 h_{s-2n} phi(2x - s)
    const int s_lo = 3 * (-p + 1), s_hi = 3 * p - 2, ns = s_hi - s_lo + 1;
    std::vector<ld> R(p * ns, 0);
    for (int k = 0; k < p; ++k)
        for (int i = 0; i < nt; ++i) {
            const int n = i - p + 1;
            for (int j = 0; j < 2 * p; ++j) {
                const int s = 2 * n + (j - p + 1);
                R[k * ns + (s - s_lo)] += 2 * Cf[i * p + k] * hk[j];
            }
        }
    const ld r2 = std::sqrt((ld)2);
    BoundaryEdge e;
    e.U.assign(p * p, 0);
    e.V.assign(p * (2 * p - 1), 0);
    std::vector<ld> Uld(p * p), Vld(p * (2 * p - 1));
    for (int k = 0; k < p; ++k) {
        for (int l = 0; l < p; ++l) {
            ld tot = 0;
            for (int si = 0; si < ns; ++si) {
                const ld bv = R[k * ns + si];
                if (bv == 0) continue;
                for (int i = 0; i < nt; ++i) tot += bv * Cf[i * p + l] * G(si + s_lo, i - p + 1);
            }
            Uld[k * p + l] = tot / r2 / r2;   // H / sqrt2, H = (1/sqrt2) sum b a G
        }
        for (int mi = 0; mi < 2 * p - 1; ++mi) {
            const int m = p + mi;
            ld tot = 0;
            for (int si = 0; si < ns; ++si) tot += R[k * ns + si] * G(si + s_lo, m);
            Vld[k * (2 * p - 1) + mi] = tot / r2 / r2;
        }
    }
    // v1(0): (I - U) v = V 1
    std::vector<ld> Am(p * p), bv(p);
    for (int k = 0; k < p; ++k) {
        ld s = 0;
        for (int mi = 0; mi < 2 * p - 1; ++mi) s += Vld[k * (2 * p - 1) + mi];
        bv[k] = s;
        for (int l = 0; l < p; ++l) Am[k * p + l] = (k == l ? 1 : 0) - Uld[k * p + l];
    }
    solve_dense(Am, bv, p);
    for (int i = 0; i < p * p; ++i) e.U[i] = (double)Uld[i];
    for (int i = 0; i < p * (2 * p - 1); ++i) e.V[i] = (double)Vld[i];
    e.v0.resize(p);
    for (int k = 0; k < p; ++k) e.v0[k] = (double)bv[k];
    e.coef.resize(nt * p);
    for (int i = 0; i < nt * p; ++i) e.coef[i] = (double)Cf[i];
    return e;
}

// phi at the integers n = -p+1..p: the fixed point of the refinement equation
// phi(n) = 2 sum_k h_k phi(2n - k) restricted to the integers, normalized by
// the partition of unity sum_n phi(n) = 1.  Haar: phi = 1 on [0, 1).
std::vector<ld> phi_at_integers(const std::vector<ld>& hk, int p) {
    if (p == 1) return {1.0L, 0.0L};
    const int n = 2 * p;   // integers -p+1..p
    std::vector<ld> A(n * n, 0), b(n, 0);
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) {
            const int k = 2 * (a - p + 1) - (c - p + 1);
            if (k >= -p + 1 && k <= p) A[a * n + c] = 2 * hk[k + p - 1];
            if (a == c) A[a * n + c] -= 1;
        }
    // the system (A - I) v = 0 has rank n - 1: replace its last row by the normalization
    for (int c = 0; c < n; ++c) A[(n - 1) * n + c] = 1;
    b[n - 1] = 1;
    solve_dense(A, b, n);
    return b;
}

}  // namespace

const BasisData& basis_data(int p) {
    static std::mutex mu;
    static std::map<int, BasisData> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(p);
    if (it != cache.end()) return it->second;
    if (p < 1 || p > 8) throw std::runtime_error("unsupported number of vanishing moments");
    BasisData d;
    d.p = p;
    const std::vector<ld> hk = daubechies_taps(p);
    d.taps.assign(hk.begin(), hk.end());
    {
        const std::vector<ld> pv = phi_at_integers(hk, p);
        d.phi_int.assign(pv.begin(), pv.end());
    }
    if (p > 1) {
        d.left = edge_construction(hk, p);
        std::vector<ld> flip(2 * p);
        for (int k = -p + 1; k <= p; ++k) flip[k + p - 1] = hk[(1 - k) + p - 1];
        d.right = edge_construction(flip, p);
    }
    return cache.emplace(p, std::move(d)).first->second;
}

namespace {

// One point: phi-hat and (optionally) both boundary vectors at eta.
struct PointEval {
    int p;
    const BasisData* bd;
    std::vector<cd> fac, dz;     // per level j=1..Ktop: m0(eta/2^j) and e^{-2 pi i eta/2^j} - 1
    std::vector<cd> sfx;         // sfx[l] = phi-hat(eta / 2^l)
    std::vector<cd> w, w2, v2;

    explicit PointEval(const BasisData* b) : p(b->p), bd(b) {}

    // m0(zeta) - 1 = sum_k h_k (z^k - 1), z = e^{-2 pi i zeta}, from d = z - 1
    cd m0_minus_one(cd d) const {
        const double* h = bd->taps.data();
        const cd z = 1.0 + d;
        cd e = d, acc = h[1 + p - 1] * e;                  // k = 1
        for (int k = 2; k <= p; ++k) { e = z * e + d; acc += h[k + p - 1] * e; }
        const cd dc = std::conj(d), zc = std::conj(z);
        e = dc;
        if (p >= 2) acc += h[-1 + p - 1] * e;              // k = -1
        for (int k = 2; k <= p - 1; ++k) { e = zc * e + dc; acc += h[-k + p - 1] * e; }
        return acc;
    }

    void run(double eta, bool boundary, cd* Lout, cd* Rout, cd& phihat) {
        const double a = std::fabs(eta);
        const int lg = (a > 1) ? (int)std::ceil(std::log2(a)) : 0;
        const int Ktop = 62 + lg;
        fac.resize(Ktop + 1);
        dz.resize(Ktop + 1);
        sfx.assign(Ktop + 1, cd(1, 0));
        double zeta = eta;
        for (int j = 1; j <= Ktop; ++j) {
            zeta *= 0.5;
            const double half = -M_PI * zeta;  // theta/2 with theta = -2 pi zeta
            const double s = std::sin(half), c = std::cos(half);
            const cd d(-2 * s * s, 2 * s * c);
            dz[j] = d;
            fac[j] = 1.0 + m0_minus_one(d);
        }
        cd acc(1, 0);
        for (int j = Ktop; j >= 1; --j) { acc *= fac[j]; sfx[j - 1] = acc; }
        phihat = sfx[0];
        if (!boundary) return;
        const int K = std::min(Ktop - 1, 36 + lg);
        const int nv = 2 * p - 1;
        w.resize(p); w2.resize(p); v2.resize(nv);
        for (int side = 0; side < 2; ++side) {
            const BoundaryEdge& E = side == 0 ? bd->left : bd->right;
            for (int k = 0; k < p; ++k) w[k] = E.v0[k];
            for (int l = K - 1; l >= 0; --l) {
                // zeta = eta / 2^{l+1}: z = e^{-2 pi i zeta} = 1 + dz[l+1]
                const cd z = 1.0 + dz[l + 1];
                const cd base = side == 0 ? z : std::conj(z);
                // left: e^{-2 pi i m zeta}, m = p..3p-2 ; right: e^{+2 pi i (m+1) zeta}
                cd pw(1, 0);
                const int first = side == 0 ? p : p + 1;
                for (int i = 0; i < first; ++i) pw *= base;
                const cd F = sfx[l + 1];
                for (int mi = 0; mi < nv; ++mi) { v2[mi] = F * pw; pw *= base; }
                for (int k = 0; k < p; ++k) {
                    cd s(0, 0);
                    for (int q = 0; q < p; ++q) s += E.U[k * p + q] * w[q];
                    const int last = std::min(nv, 2 * k + 1);   // staircase of V
                    for (int mi = 0; mi < last; ++mi) s += E.V[k * nv + mi] * v2[mi];
                    w2[k] = s;
                }
                std::swap(w, w2);
            }
            cd* out = side == 0 ? Lout : Rout;
            for (int k = 0; k < p; ++k) out[k] = w[k];
        }
    }
};

}  // namespace

void eval_basis_1d(int J, int p, int64_t M, const double* xi, int stride, cd* out, int nthreads) {
    const BasisData& bd = basis_data(p);
    const int nb = (p == 1) ? 0 : p;
    const int nch = 2 * nb + 1;
    const double scale = std::ldexp(1.0, 0) / std::sqrt(std::ldexp(1.0, J));
    auto work = [&](int64_t b, int64_t e) {
        PointEval pe(&bd);
        std::vector<cd> Lv(p), Rv(p);
        for (int64_t m = b; m < e; ++m) {
            const double x = xi[m * stride];
            const double eta = std::ldexp(x, -J);
            cd ph;
            pe.run(eta, nb > 0, Lv.data(), Rv.data(), ph);
            cd* o = out + m * nch;
            o[nb] = scale * ph;
            if (nb) {
                const double r = std::fmod(x, 2.0);    // exact
                const cd e_plus(std::cos(M_PI * r), std::sin(M_PI * r));
                for (int c = 0; c < nb; ++c) {
                    o[c] = scale * e_plus * Lv[c];
                    o[nb + 1 + c] = scale * std::conj(e_plus) * Rv[c];
                }
            }
        }
    };
    if (nthreads <= 1 || M < 4096) {
        work(0, M);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (M + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        const int64_t b = t * chunk, e = std::min<int64_t>(M, b + chunk);
        if (b < e) th.emplace_back(work, b, e);
    }
    for (auto& t : th) t.join();
}

// ---------------------------------------------------------------- KB window

namespace {
ld bessel_i0(ld x) {
    const ld q = x * x / 4;
    ld term = 1, sum = 1;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((ld)k * (ld)k);
        sum += term;
        if (term < sum * 1e-21L) break;
    }
    return sum;
}
}  // namespace

double KBWindow::eval_exact(double d) const {
    const ld z = 1 - (2 * (ld)d / w) * (2 * (ld)d / w);
    if (z < 0) return 0;
    return (double)(bessel_i0(beta * std::sqrt(z)) / bessel_i0(beta));
}

double KBWindow::ft(double f) const {
    const ld a = (ld)beta * beta - (M_PI * (ld)w * f) * (M_PI * (ld)w * f);
    ld v;
    if (a > 0) {
        const ld s = std::sqrt(a);
        v = w * std::sinh(s) / s;
    } else if (a < 0) {
        const ld s = std::sqrt(-a);
        v = w * std::sin(s) / s;
    } else {
        v = w;
    }
    return (double)(v / bessel_i0(beta));
}

KBWindow make_window(int w, int deg, double beta) {
    KBWindow kb;
    kb.w = w;
    kb.deg = deg;
    kb.beta = beta;
    const int n = deg + 1;
    kb.coef.assign(w * n, 0);
    const ld i0b = bessel_i0(beta);
    for (int j = 0; j < w; ++j) {
        std::vector<ld> f(n), c(n, 0);
        for (int i = 0; i < n; ++i) {
            const ld x = std::cos(M_PI * (i + 0.5L) / n);
            const ld d = (x + 1) / 2 + (ld)w / 2 - 1 - j;
            const ld z = 1 - (2 * d / w) * (2 * d / w);
            f[i] = z < 0 ? 0 : bessel_i0(beta * std::sqrt(z)) / i0b;
        }
        for (int k = 0; k < n; ++k) {
            ld s = 0;
            for (int i = 0; i < n; ++i) s += f[i] * std::cos(M_PI * k * (i + 0.5L) / n);
            c[k] = 2 * s / n;
        }
        c[0] /= 2;
        // Chebyshev -> monomial: T_0 = 1, T_1 = x, T_{k+1} = 2x T_k - T_{k-1}
        std::vector<ld> tkm1(n, 0), tk(n, 0), a(n, 0);
        tkm1[0] = 1;
        if (n > 1) tk[1] = 1;
        for (int i = 0; i < n; ++i) a[i] += c[0] * tkm1[i];
        if (n > 1)
            for (int i = 0; i < n; ++i) a[i] += c[1] * tk[i];
        for (int k = 2; k < n; ++k) {
            std::vector<ld> tn(n, 0);
            for (int i = 0; i < n - 1; ++i) tn[i + 1] += 2 * tk[i];
            for (int i = 0; i < n; ++i) tn[i] -= tkm1[i];
            for (int i = 0; i < n; ++i) a[i] += c[k] * tn[i];
            tkm1 = tk;
            tk = tn;
        }
        for (int i = 0; i < n; ++i) kb.coef[j * n + i] = (double)a[i];
    }
    return kb;
}

}  // namespace gs
