// Sum-of-exponentials (SOE) tables of the Gaussian (host, FP64).
//
// The SOE of Sec. 3 (eq. SOE1), e^{-x^2} ~ sum_l w_l e^{-s_l |x|}, turns every
// Fourier mode's pair kernel into exponentials of |z_i - z_j| (eq. SOEphi), so
// that each mode costs O(N) through the z-ordered recursion; the number of
// terms M sets the cost of every k != 0 and k = 0 pass.  Tables are closed
// under complex conjugation with Re s_l > 0.  Two constructions:
//
//  * q2d_soe_fit: the midpoint rule on Weideman's optimised Talbot contour of
//    the inverse-Laplace representation
//        e^{-x^2} = (1/2 pi i) int e^z sqrt(pi/z) e^{-2 sqrt(z) |x|} dz
//    (the printed form has e^{-sqrt(z)|x|}; the Laplace pair
//    e^{-a sqrt(p)}/sqrt(p) <-> e^{-a^2/4t}/sqrt(pi t) at t = 1 fixes the
//    factor 2), with the contour scale of smallest sup error;
//
//  * q2d_soe_fit_reduced: model reduction, which the paper's VPMR tables rely
//    on as well (it does not list them).  A Talbot SOE with many terms is the
//    impulse response h(x) = C e^{A x} B of a linear system with
//    A = -diag(s_l), B_l = C_l = sqrt(w_l).  Square-root balanced truncation
//    keeps the M states of largest Hankel singular value (the discarded ones
//    bound the error); the poles of the reduced system are the new exponents
//    (conjugate pairs), the weights follow by linear least squares on a grid,
//    and a Lawson-weighted Levenberg-Marquardt polish moves the whole table
//    toward the minimax one.  M = 10 reaches the sup error that the Talbot
//    rule needs M = 16 for (about 7e-10).
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "q2d_internal.h"

namespace {

using cd = std::complex<double>;
const double PI = 3.14159265358979323846;

struct Fit {
    std::vector<cd> w, s;
};

// Midpoint rule on Weideman's optimised Talbot contour
//   z(t) = n (sigma + mu t cot(a t) + i nu t), t in (-pi, pi).
Fit talbot(int M, double scale) {
    const double sg = -0.6122, mu = 0.5017, a = 0.6407, nu = 0.2645;
    const double h = 2.0 * PI / M, n = M * scale;
    Fit f;
    for (int j = 0; j < M; ++j) {
        const double t = -PI + (j + 0.5) * h;
        const cd z = n * cd(sg + mu * t / std::tan(a * t), nu * t);
        const double st = std::sin(a * t);
        const cd dz = n * cd(mu * (1.0 / std::tan(a * t) - a * t / (st * st)), nu);
        const cd w = h / (2.0 * PI * cd(0, 1)) * std::exp(z) * std::sqrt(PI / z) * dz;
        f.w.push_back(w);
        f.s.push_back(2.0 * std::sqrt(z));
    }
    return f;
}

// max |e^{-x^2} - SOE(x)| on a grid: dense on [0, 12], sparse on [12, 200]
double sup_err(const Fit &f, int npts) {
    double e = 0.0;
    for (int i = 0; i <= npts; ++i) {
        const double x = i < npts * 9 / 10 ? 12.0 * i / (npts * 9 / 10)
                                           : 12.0 + 188.0 * (i - npts * 9 / 10) / (npts / 10);
        cd v = 0.0;
        for (size_t l = 0; l < f.w.size(); ++l) v += f.w[l] * std::exp(-f.s[l] * x);
        e = std::max(e, std::fabs(v.real() - std::exp(-x * x)));
    }
    return e;
}

Fit best_talbot(int M) {
    Fit best;
    double be = 1e300;
    for (int i = 0; i <= 40; ++i) {
        Fit f = talbot(M, 0.6 + 0.02 * i);
        const double e = sup_err(f, 4000);
        if (e < be) {
            be = e;
            best = f;
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// small dense complex linear algebra
// ---------------------------------------------------------------------------
struct CMat {
    int r = 0, c = 0;
    std::vector<cd> a;
    CMat() = default;
    CMat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, cd(0.0, 0.0)) {}
    cd &operator()(int i, int j) { return a[(size_t)i * c + j]; }
    const cd &operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

// Pivoted Cholesky of a Hermitian positive semidefinite matrix: P ~ L L^H with
// L of n x k, stopping when the largest remaining pivot falls below tol times
// the largest diagonal entry (the Gramians below are numerically singular).
CMat pivoted_cholesky(const CMat &P, double tol) {
    const int n = P.r;
    CMat A = P, L(n, n);
    std::vector<int> piv(n);
    std::iota(piv.begin(), piv.end(), 0);
    double d0 = 0.0;
    for (int i = 0; i < n; ++i) d0 = std::max(d0, A(i, i).real());
    int k = 0;
    for (; k < n; ++k) {
        int jm = k;
        for (int j = k + 1; j < n; ++j)
            if (A(piv[j], piv[j]).real() > A(piv[jm], piv[jm]).real()) jm = j;
        const double dm = A(piv[jm], piv[jm]).real();
        if (!(dm > tol * d0)) break;
        std::swap(piv[k], piv[jm]);
        const int p = piv[k];
        const double d = std::sqrt(dm);
        for (int jj = k; jj < n; ++jj) L(piv[jj], k) = A(piv[jj], p) / d;
        for (int a = k + 1; a < n; ++a)
            for (int b = k + 1; b < n; ++b)
                A(piv[a], piv[b]) -= L(piv[a], k) * std::conj(L(piv[b], k));
    }
    CMat R(n, k);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) R(i, j) = L(i, j);
    return R;
}

// One-sided (Hestenes) Jacobi SVD: G = U diag(sig) V^H, singular values in
// decreasing order (U: m x n, V: n x n).
void jacobi_svd(CMat G, std::vector<double> &sig, CMat &U, CMat &V) {
    const int m = G.r, n = G.c;
    V = CMat(n, n);
    for (int i = 0; i < n; ++i) V(i, i) = 1.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double a = 0.0, b = 0.0;
                cd g = 0.0;
                for (int k = 0; k < m; ++k) {
                    a += std::norm(G(k, i));
                    b += std::norm(G(k, j));
                    g += std::conj(G(k, i)) * G(k, j);
                }
                const double ag = std::abs(g);
                if (ag == 0.0 || ag <= 1e-15 * std::sqrt(a * b)) continue;
                off = std::max(off, ag / std::sqrt(a * b));
                // phase column j so that the pair's inner product is real, then
                // rotate the pair as the real symmetric Jacobi method does
                const cd ph = std::conj(g / ag);
                const double zeta = (b - a) / (2.0 * ag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int k = 0; k < m; ++k) {
                    const cd x = G(k, i), y = G(k, j) * ph;
                    G(k, i) = c * x - s * y;
                    G(k, j) = s * x + c * y;
                }
                for (int k = 0; k < n; ++k) {
                    const cd x = V(k, i), y = V(k, j) * ph;
                    V(k, i) = c * x - s * y;
                    V(k, j) = s * x + c * y;
                }
            }
        if (off < 1e-14) break;
    }
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) {
        double a = 0.0;
        for (int k = 0; k < m; ++k) a += std::norm(G(k, j));
        nrm[j] = std::sqrt(a);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    sig.assign(n, 0.0);
    CMat Us(m, n), Vs(n, n);
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        sig[jj] = nrm[j];
        for (int k = 0; k < m; ++k) Us(k, jj) = nrm[j] > 0 ? G(k, j) / nrm[j] : cd(0.0, 0.0);
        for (int k = 0; k < n; ++k) Vs(k, jj) = V(k, j);
    }
    U = Us;
    V = Vs;
}

// Eigenvalues of a small complex matrix: Householder reduction to Hessenberg
// form, then single-shift QR steps (Wilkinson shift, Givens rotations) on the
// active block with deflation at negligible subdiagonal entries.
bool eigenvalues(CMat H, std::vector<cd> &ev) {
    const int n = H.r;
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<cd> v(len);
        double xn = 0.0;
        for (int i = 0; i < len; ++i) {
            v[i] = H(k + 1 + i, k);
            xn += std::norm(v[i]);
        }
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const cd ph = std::abs(v[0]) > 0 ? v[0] / std::abs(v[0]) : cd(1.0, 0.0);
        v[0] += ph * xn;
        double vn = 0.0;
        for (int i = 0; i < len; ++i) vn += std::norm(v[i]);
        vn = std::sqrt(vn);
        for (int i = 0; i < len; ++i) v[i] /= vn;
        for (int j = 0; j < n; ++j) {  // H = (I - 2 v v^H) H
            cd w = 0.0;
            for (int i = 0; i < len; ++i) w += std::conj(v[i]) * H(k + 1 + i, j);
            for (int i = 0; i < len; ++i) H(k + 1 + i, j) -= 2.0 * v[i] * w;
        }
        for (int i = 0; i < n; ++i) {  // H = H (I - 2 v v^H)
            cd w = 0.0;
            for (int j = 0; j < len; ++j) w += H(i, k + 1 + j) * v[j];
            for (int j = 0; j < len; ++j) H(i, k + 1 + j) -= 2.0 * w * std::conj(v[j]);
        }
    }
    ev.clear();
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) {
            ev.push_back(H(0, 0));
            break;
        }
        int l = hi;
        while (l > 0 && std::abs(H(l, l - 1)) >
                            1e-15 * (std::abs(H(l, l)) + std::abs(H(l - 1, l - 1))))
            --l;
        if (l == hi) {
            ev.push_back(H(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 500) return false;
        const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
        const cd tr = a + d, disc = std::sqrt(tr * tr / 4.0 - (a * d - b * c));
        const cd m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
        cd mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        if (iter % 11 == 10) mu += std::abs(H(hi, hi - 1));  // exceptional shift
        for (int i = l; i <= hi; ++i) H(i, i) -= mu;
        std::vector<cd> gc(hi - l), gs(hi - l);
        for (int k = l; k < hi; ++k) {
            const cd x = H(k, k), y = H(k + 1, k);
            const double r = std::hypot(std::abs(x), std::abs(y));
            const cd cs = r > 0 ? x / r : cd(1.0, 0.0), sn = r > 0 ? y / r : cd(0.0, 0.0);
            gc[k - l] = cs;
            gs[k - l] = sn;
            for (int j = l; j <= hi; ++j) {  // rows k, k+1 <- G rows
                const cd u = H(k, j), w = H(k + 1, j);
                H(k, j) = std::conj(cs) * u + std::conj(sn) * w;
                H(k + 1, j) = -sn * u + cs * w;
            }
        }
        for (int k = l; k < hi; ++k) {  // columns k, k+1 <- columns G^H
            const cd cs = gc[k - l], sn = gs[k - l];
            for (int i = l; i <= hi; ++i) {
                const cd u = H(i, k), w = H(i, k + 1);
                H(i, k) = u * cs + w * sn;
                H(i, k + 1) = -u * std::conj(sn) + w * std::conj(cs);
            }
        }
        for (int i = l; i <= hi; ++i) H(i, i) += mu;
    }
    return (int)ev.size() == n;
}

// Real linear least squares min ||A x - b|| (A: m x n, row-major) by
// Householder QR.
bool lsq(std::vector<double> A, std::vector<double> b, int m, int n, std::vector<double> &x) {
    for (int k = 0; k < n; ++k) {
        double xn = 0.0;
        for (int i = k; i < m; ++i) xn += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        xn = std::sqrt(xn);
        if (xn == 0.0) return false;
        const double alpha = A[(size_t)k * n + k] > 0 ? -xn : xn;
        std::vector<double> v(m - k);
        for (int i = k; i < m; ++i) v[i - k] = A[(size_t)i * n + k];
        v[0] -= alpha;
        double vn = 0.0;
        for (double t : v) vn += t * t;
        if (vn == 0.0) continue;
        for (int j = k; j < n; ++j) {
            double w = 0.0;
            for (int i = k; i < m; ++i) w += v[i - k] * A[(size_t)i * n + j];
            w *= 2.0 / vn;
            for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= w * v[i - k];
        }
        double w = 0.0;
        for (int i = k; i < m; ++i) w += v[i - k] * b[i];
        w *= 2.0 / vn;
        for (int i = k; i < m; ++i) b[i] -= w * v[i - k];
    }
    x.assign(n, 0.0);
    for (int k = n - 1; k >= 0; --k) {
        double t = b[k];
        for (int j = k + 1; j < n; ++j) t -= A[(size_t)k * n + j] * x[j];
        if (A[(size_t)k * n + k] == 0.0) return false;
        x[k] = t / A[(size_t)k * n + k];
    }
    return true;
}

// Cholesky solve of a symmetric positive definite system (in place)
bool chol_solve(std::vector<double> A, std::vector<double> &b, int n) {
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / d;
        }
    }
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * b[k];
        b[i] = t / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < n; ++k) t -= A[(size_t)k * n + i] * b[k];
        b[i] = t / A[(size_t)i * n + i];
    }
    return true;
}

// fitting grid: dense where the Gaussian lives, sparse in the tail
std::vector<double> fit_grid() {
    std::vector<double> x;
    for (int i = 0; i < 3000; ++i) x.push_back(6.5 * i / 2999.0);
    for (int i = 1; i <= 400; ++i) x.push_back(6.5 + 33.5 * i / 400.0);
    return x;
}

// A table from pair representatives (Im s > 0): value 2 Re sum_p w_p e^{-s_p x}
Fit from_pairs(const std::vector<cd> &w, const std::vector<cd> &s) {
    Fit f;
    for (size_t p = 0; p < w.size(); ++p) {
        f.w.push_back(w[p]);
        f.s.push_back(s[p]);
    }
    for (size_t p = 0; p < w.size(); ++p) {
        f.w.push_back(std::conj(w[p]));
        f.s.push_back(std::conj(s[p]));
    }
    return f;
}

// weights of fixed pair exponents by least squares on the grid
bool pair_weights(const std::vector<cd> &s, const std::vector<double> &x, std::vector<cd> &w) {
    const int h = (int)s.size(), m = (int)x.size(), n = 2 * h;
    std::vector<double> A((size_t)m * n), b(m), c;
    for (int i = 0; i < m; ++i) {
        for (int p = 0; p < h; ++p) {
            const cd e = std::exp(-s[p] * x[i]);
            A[(size_t)i * n + p] = 2.0 * e.real();
            A[(size_t)i * n + h + p] = -2.0 * e.imag();
        }
        b[i] = std::exp(-x[i] * x[i]);
    }
    if (!lsq(A, b, m, n, c)) return false;
    w.resize(h);
    for (int p = 0; p < h; ++p) w[p] = cd(c[p], c[h + p]);
    return true;
}

// Levenberg-Marquardt on (w_p, s_p) for the weighted residual on the grid,
// with Lawson reweighting (weights grow where the error is largest) every 10
// iterations; keeps the table of smallest grid sup error.
void polish(std::vector<cd> &w, std::vector<cd> &s, const std::vector<double> &x, int iters) {
    const int h = (int)w.size(), m = (int)x.size(), n = 4 * h;
    std::vector<double> wt(m, 1.0), f(m);
    for (int i = 0; i < m; ++i) f[i] = std::exp(-x[i] * x[i]);
    auto value = [&](const std::vector<cd> &ww, const std::vector<cd> &ss, std::vector<double> &g) {
        g.assign(m, 0.0);
        for (int i = 0; i < m; ++i) {
            cd v = 0.0;
            for (int p = 0; p < h; ++p) v += ww[p] * std::exp(-ss[p] * x[i]);
            g[i] = 2.0 * v.real();
        }
    };
    auto cost = [&](const std::vector<double> &g) {
        double c = 0.0;
        for (int i = 0; i < m; ++i) c += (wt[i] * (g[i] - f[i])) * (wt[i] * (g[i] - f[i]));
        return c;
    };
    auto supg = [&](const std::vector<double> &g) {
        double e = 0.0;
        for (int i = 0; i < m; ++i) e = std::max(e, std::fabs(g[i] - f[i]));
        return e;
    };
    std::vector<double> g;
    value(w, s, g);
    double c0 = cost(g), best_e = supg(g), lam = 1e-3;
    std::vector<cd> bw = w, bs = s;
    int since = 0;
    std::vector<double> J((size_t)n), JtJ((size_t)n * n), Jtr(n);
    for (int it = 0; it < iters; ++it) {
        std::fill(JtJ.begin(), JtJ.end(), 0.0);
        std::fill(Jtr.begin(), Jtr.end(), 0.0);
        for (int i = 0; i < m; ++i) {
            for (int p = 0; p < h; ++p) {
                const cd e = std::exp(-s[p] * x[i]);
                const cd we = w[p] * e * x[i];
                J[p] = 2.0 * e.real();
                J[h + p] = -2.0 * e.imag();
                J[2 * h + p] = -2.0 * we.real();
                J[3 * h + p] = 2.0 * we.imag();
            }
            const double r = wt[i] * (g[i] - f[i]);
            for (int a = 0; a < n; ++a) {
                const double ja = wt[i] * J[a];
                Jtr[a] += ja * r;
                for (int b = 0; b <= a; ++b) JtJ[(size_t)a * n + b] += ja * wt[i] * J[b];
            }
        }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < a; ++b) JtJ[(size_t)b * n + a] = JtJ[(size_t)a * n + b];
        bool stepped = false;
        while (lam < 1e10) {
            std::vector<double> A = JtJ, d(n);
            for (int a = 0; a < n; ++a) {
                A[(size_t)a * n + a] += lam * (JtJ[(size_t)a * n + a] + 1e-300);
                d[a] = -Jtr[a];
            }
            if (chol_solve(A, d, n)) {
                std::vector<cd> w2(h), s2(h);
                bool ok = true;
                for (int p = 0; p < h; ++p) {
                    w2[p] = w[p] + cd(d[p], d[h + p]);
                    s2[p] = s[p] + cd(d[2 * h + p], d[3 * h + p]);
                    if (!(s2[p].real() > 0) || !(s2[p].imag() > 0)) ok = false;
                }
                if (ok) {
                    std::vector<double> g2;
                    value(w2, s2, g2);
                    const double c2 = cost(g2);
                    if (c2 < c0) {
                        w = w2;
                        s = s2;
                        g = g2;
                        c0 = c2;
                        lam = std::max(lam / 3.0, 1e-12);
                        stepped = true;
                        break;
                    }
                }
            }
            lam *= 4.0;
        }
        if (!stepped) break;
        const double e = supg(g);
        if (e < best_e * (1.0 - 1e-3)) {
            best_e = e;
            bw = w;
            bs = s;
            since = 0;
        } else if (e < best_e) {
            best_e = e;
            bw = w;
            bs = s;
            ++since;
        } else {
            ++since;
        }
        if (since > 300) break;
        if (it % 10 == 9) {
            double mx = 0.0;
            for (int i = 0; i < m; ++i) mx = std::max(mx, std::fabs(g[i] - f[i]));
            double wm = 0.0;
            for (int i = 0; i < m; ++i) {
                wt[i] *= std::sqrt(std::max(std::fabs(g[i] - f[i]) / mx, 1e-3));
                wm = std::max(wm, wt[i]);
            }
            for (int i = 0; i < m; ++i) wt[i] /= wm;
            c0 = cost(g);
        }
    }
    w = bw;
    s = bs;
}

// Model-reduced M-term table (M even): balanced truncation of the 48-term
// Talbot SOE, least-squares weights, polish.
bool reduced_fit(int M, Fit &out) {
    const Fit ref = best_talbot(48);
    const int n = (int)ref.w.size(), r = M;
    std::vector<cd> B(n), C(n);
    for (int l = 0; l < n; ++l) {
        B[l] = std::sqrt(ref.w[l]);
        C[l] = ref.w[l] / B[l];
    }
    // Gramians of x' = A x + B u, y = C x with A = -diag(s):
    //   P_ij = B_i conj(B_j) / (s_i + conj(s_j)),  Q_ij = conj(C_i) C_j / (conj(s_i) + s_j)
    CMat P(n, n), Q(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            P(i, j) = B[i] * std::conj(B[j]) / (ref.s[i] + std::conj(ref.s[j]));
            Q(i, j) = std::conj(C[i]) * C[j] / (std::conj(ref.s[i]) + ref.s[j]);
        }
    const CMat Lp = pivoted_cholesky(P, 1e-30), Lq = pivoted_cholesky(Q, 1e-30);
    if (Lp.c < r || Lq.c < r) return false;
    CMat G(Lq.c, Lp.c);  // Lq^H Lp
    for (int a = 0; a < Lq.c; ++a)
        for (int b = 0; b < Lp.c; ++b) {
            cd t = 0.0;
            for (int i = 0; i < n; ++i) t += std::conj(Lq(i, a)) * Lp(i, b);
            G(a, b) = t;
        }
    std::vector<double> sig;
    CMat U, V;
    jacobi_svd(G, sig, U, V);
    if ((int)sig.size() < r || !(sig[r - 1] > 0)) return false;
    // T = Lp V_r S^{-1/2}, Ti = S^{-1/2} U_r^H Lq^H, A_r = Ti A T
    CMat T(n, r), Ti(r, n), Ar(r, r);
    for (int i = 0; i < n; ++i)
        for (int b = 0; b < r; ++b) {
            cd t = 0.0;
            for (int k = 0; k < Lp.c; ++k) t += Lp(i, k) * V(k, b);
            T(i, b) = t / std::sqrt(sig[b]);
        }
    for (int a = 0; a < r; ++a)
        for (int i = 0; i < n; ++i) {
            cd t = 0.0;
            for (int k = 0; k < Lq.c; ++k) t += std::conj(U(k, a)) * std::conj(Lq(i, k));
            Ti(a, i) = t / std::sqrt(sig[a]);
        }
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
            cd t = 0.0;
            for (int i = 0; i < n; ++i) t += Ti(a, i) * (-ref.s[i]) * T(i, b);
            Ar(a, b) = t;
        }
    std::vector<cd> lam;
    if (!eigenvalues(Ar, lam)) return false;
    // exponents s = -lambda: a real system's poles come in conjugate pairs;
    // keep the r/2 with the largest imaginary part as representatives
    std::vector<cd> sp;
    for (cd l : lam) sp.push_back(-l);
    std::sort(sp.begin(), sp.end(), [](cd a, cd b) { return a.imag() > b.imag(); });
    sp.resize(r / 2);
    for (cd v : sp)
        if (!(v.real() > 0) || !(v.imag() > 1e-8 * std::abs(v))) return false;
    const std::vector<double> x = fit_grid();
    std::vector<cd> wp;
    if (!pair_weights(sp, x, wp)) return false;
    polish(wp, sp, x, 1500);
    out = from_pairs(wp, sp);
    return true;
}

void put(const Fit &f, double *w, double *s) {
    for (size_t l = 0; l < f.w.size(); ++l) {
        w[2 * l] = f.w[l].real();
        w[2 * l + 1] = f.w[l].imag();
        s[2 * l] = f.s[l].real();
        s[2 * l + 1] = f.s[l].imag();
    }
}

}  // namespace

extern "C" {

q2d_status q2d_soe_fit(int32_t M, double *w, double *s, double *sup_error) {
    if (!w || !s || M < 2 || M > 64 || (M % 2)) return Q2D_EINVAL;
    const Fit best = best_talbot(M);
    put(best, w, s);
    if (sup_error) *sup_error = sup_err(best, 40000);
    return Q2D_OK;
}

q2d_status q2d_soe_fit_reduced(int32_t M, double *w, double *s, double *sup_error) {
    if (!w || !s || M < 2 || M > Q2D_SOE_REDUCED_MAX || (M % 2)) return Q2D_EINVAL;
    Fit f;
    if (!reduced_fit(M, f)) return Q2D_EUNSUPPORTED;
    put(f, w, s);
    if (sup_error) *sup_error = sup_err(f, 40000);
    return Q2D_OK;
}

q2d_status q2d_soe_fit_eps(double eps, int32_t M_max, int32_t *M, double *w, double *s,
                           double *sup_error) {
    if (!M || !w || !s || !(eps > 0) || M_max < 2 || M_max > 64) return Q2D_EINVAL;
    for (int m = 2; m <= M_max; m += 2) {
        Fit f = best_talbot(m);
        double e = sup_err(f, 40000);
        Fit fr;
        if (m <= Q2D_SOE_REDUCED_MAX && reduced_fit(m, fr)) {
            const double er = sup_err(fr, 40000);
            if (er < e) {
                f = fr;
                e = er;
            }
        }
        put(f, w, s);
        *M = m;
        if (sup_error) *sup_error = e;
        if (e <= eps) return Q2D_OK;
    }
    return Q2D_ECAPACITY;
}

}  // extern "C"
