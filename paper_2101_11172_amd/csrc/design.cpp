// Host-side least-misfit kernel design and planner (float64).
//
// The error bound E (eq. norm_bound) is minimised over the correction h and the
// gridding function C.  For a fixed h the best C at each nu is the solution of a
// W x W linear least-squares problem (normal matrix A, right-hand side b(nu));
// eliminating C this way leaves a nonlinear least-squares problem in h alone,
// solved by Levenberg-Marquardt on the values of h at Gauss-Legendre nodes, with
// the residuals L(x, nu) of eq. csum2 at the node pairs.  Jacobians come from the
// complex step (every operation on h is analytic: products, sums and an LDL^T
// solve without pivoting of the positive-definite A).  The start is the
// Kaiser-Bessel kernel with the best shape parameter on a scan.
#include "design.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>

namespace wsg {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kNodes = 32;        // Gauss-Legendre nodes in x and in nu
constexpr int kDegree = 16;       // per-segment polynomial degree in nu, float64 path
constexpr int kDegreeLo = 8;      // float32 path: fit error ~1e-9 of max |C|, below float32 rounding

void gauss_legendre(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[n - 1 - i] = 0.5 * (b - a) * t + 0.5 * (b + a);
        w[n - 1 - i] = (b - a) / ((1.0 - t * t) * dp * dp);
    }
}

// Modified Bessel function I0 by its power series (all terms positive).
double bessel_i0(double x) {
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// In-place LDL^T solve of the symmetric positive-definite n x n system M y = rhs
// for `nrhs` right-hand sides stored as rhs[r*n + i]; no pivoting (analytic in M).
template <class T>
void ldlt_solve(int n, std::vector<T>& M, T* rhs, int nrhs) {
    for (int j = 0; j < n; ++j) {
        for (int k = 0; k < j; ++k) M[j * n + j] -= M[j * n + k] * M[j * n + k] * M[k * n + k];
        for (int i = j + 1; i < n; ++i) {
            T s = M[i * n + j];
            for (int k = 0; k < j; ++k) s -= M[i * n + k] * M[j * n + k] * M[k * n + k];
            M[i * n + j] = s / M[j * n + j];
        }
    }
    for (int r = 0; r < nrhs; ++r) {
        T* y = rhs + r * n;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < i; ++k) y[i] -= M[i * n + k] * y[k];
        for (int i = 0; i < n; ++i) y[i] /= M[i * n + i];
        for (int i = n - 1; i >= 0; --i)
            for (int k = i + 1; k < n; ++k) y[i] -= M[k * n + i] * y[k];
    }
}

struct Problem {
    int W, nx, nn;
    double x0;
    std::vector<double> s, xn, wx, nun, wn;
    std::vector<double> cosv, sinv;   // [nn][W][nx]  cos/sin(2 pi (s - nu) x)
    std::vector<double> K;            // [W][W][nx]   cos(2 pi (s - s') x)
    std::vector<double> sw;           // [nn][nx]     sqrt(wn wx / x0)

    Problem(int W_, double x0_) : W(W_), nx(kNodes), nn(kNodes), x0(x0_) {
        s.resize(W);
        for (int a = 0; a < W; ++a) s[a] = a - 0.5 * (W - 1);
        gauss_legendre(nx, 0.0, x0, xn, wx);
        gauss_legendre(nn, -0.5, 0.5, nun, wn);
        cosv.resize(size_t(nn) * W * nx);
        sinv.resize(size_t(nn) * W * nx);
        for (int j = 0; j < nn; ++j)
            for (int a = 0; a < W; ++a)
                for (int i = 0; i < nx; ++i) {
                    double ang = 2.0 * kPi * (s[a] - nun[j]) * xn[i];
                    cosv[(size_t(j) * W + a) * nx + i] = std::cos(ang);
                    sinv[(size_t(j) * W + a) * nx + i] = std::sin(ang);
                }
        K.resize(size_t(W) * W * nx);
        for (int a = 0; a < W; ++a)
            for (int b = 0; b < W; ++b)
                for (int i = 0; i < nx; ++i)
                    K[(size_t(a) * W + b) * nx + i] = std::cos(2.0 * kPi * (s[a] - s[b]) * xn[i]);
        sw.resize(size_t(nn) * nx);
        for (int j = 0; j < nn; ++j)
            for (int i = 0; i < nx; ++i) sw[j * nx + i] = std::sqrt(wn[j] * wx[i] / x0);
    }

    // Best c at the nu nodes for the given h: out[j*W + a].
    template <class T>
    void best_c(const T* h, std::vector<T>& c) const {
        std::vector<T> A(size_t(W) * W, T(0));
        for (int a = 0; a < W; ++a)
            for (int b = 0; b < W; ++b) {
                T acc(0);
                for (int i = 0; i < nx; ++i) acc += K[(size_t(a) * W + b) * nx + i] * (h[i] * h[i] * wx[i]);
                A[a * W + b] = acc;
            }
        c.assign(size_t(nn) * W, T(0));
        for (int j = 0; j < nn; ++j)
            for (int a = 0; a < W; ++a) {
                T acc(0);
                for (int i = 0; i < nx; ++i) acc += cosv[(size_t(j) * W + a) * nx + i] * (h[i] * wx[i]);
                c[j * W + a] = acc;
            }
        ldlt_solve(W, A, c.data(), nn);
    }

    // Weighted residuals L at the (nu, x) nodes, real parts then imaginary parts.
    template <class T>
    void residuals(const T* h, T* r) const {
        std::vector<T> c;
        best_c(h, c);
        for (int j = 0; j < nn; ++j)
            for (int i = 0; i < nx; ++i) {
                T gr(0), gi(0);
                for (int a = 0; a < W; ++a) {
                    gr += c[j * W + a] * cosv[(size_t(j) * W + a) * nx + i];
                    gi += c[j * W + a] * sinv[(size_t(j) * W + a) * nx + i];
                }
                r[j * nx + i] = (1.0 - h[i] * gr) * sw[j * nx + i];
                r[nn * nx + j * nx + i] = -(h[i] * gi) * sw[j * nx + i];
            }
    }

    double sumsq(const std::vector<double>& h) const {
        std::vector<double> r(size_t(2) * nn * nx);
        residuals(h.data(), r.data());
        double f = 0;
        for (double v : r) f += v * v;
        return f;
    }

    // Pointwise-optimal h at the x nodes for given c at the nu nodes.
    void h_from_c(const std::vector<double>& c, std::vector<double>& h) const {
        h.assign(nx, 0.0);
        for (int i = 0; i < nx; ++i) {
            double num = 0, den = 0;
            for (int j = 0; j < nn; ++j) {
                double gr = 0, gi = 0;
                for (int a = 0; a < W; ++a) {
                    gr += c[j * W + a] * cosv[(size_t(j) * W + a) * nx + i];
                    gi += c[j * W + a] * sinv[(size_t(j) * W + a) * nx + i];
                }
                num += wn[j] * gr;
                den += wn[j] * (gr * gr + gi * gi);
            }
            h[i] = num / den;
        }
    }
};

// Least squares min |J d + r|^2 + lam |d|^2 by Householder QR of [J; sqrt(lam) I].
// J is m x n column-major.
std::vector<double> damped_lstsq(const std::vector<double>& J, const std::vector<double>& r, int m,
                                 int n, double lam) {
    int mm = m + n;
    std::vector<double> Q(size_t(mm) * n, 0.0), y(mm, 0.0);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < m; ++i) Q[size_t(c) * mm + i] = J[size_t(c) * m + i];
        Q[size_t(c) * mm + m + c] = std::sqrt(lam);
    }
    for (int i = 0; i < m; ++i) y[i] = -r[i];
    for (int k = 0; k < n; ++k) {
        double* col = &Q[size_t(k) * mm];
        double norm = 0;
        for (int i = k; i < mm; ++i) norm += col[i] * col[i];
        norm = std::sqrt(norm);
        if (norm == 0) continue;
        double alpha = col[k] > 0 ? -norm : norm;
        std::vector<double> v(col + k, col + mm);
        v[0] -= alpha;
        double vn = 0;
        for (double e : v) vn += e * e;
        if (vn == 0) continue;
        for (int c = k; c < n; ++c) {
            double* cc = &Q[size_t(c) * mm];
            double dot = 0;
            for (int i = k; i < mm; ++i) dot += v[i - k] * cc[i];
            double f = 2.0 * dot / vn;
            for (int i = k; i < mm; ++i) cc[i] -= f * v[i - k];
        }
        double dot = 0;
        for (int i = k; i < mm; ++i) dot += v[i - k] * y[i];
        double f = 2.0 * dot / vn;
        for (int i = k; i < mm; ++i) y[i] -= f * v[i - k];
    }
    std::vector<double> d(n, 0.0);
    for (int k = n - 1; k >= 0; --k) {
        double s = y[k];
        for (int c = k + 1; c < n; ++c) s -= Q[size_t(c) * mm + k] * d[c];
        double diag = Q[size_t(k) * mm + k];
        d[k] = diag != 0 ? s / diag : 0.0;
    }
    return d;
}

// Per-segment polynomial in nu of degree Dg: interpolate c at Dg+1 Chebyshev
// points of [-1/2, 1/2], then convert the Chebyshev series (in t = 2 nu) to
// monomials in nu.  Returns [W][Dg+1].
std::vector<double> fit_segments(const KernelDesign& D, int Dg) {
    const int W = D.W, np = Dg + 1;
    std::vector<double> out(size_t(W) * np, 0.0), vals(size_t(np) * W);
    for (int k = 0; k < np; ++k) {
        double t = std::cos(kPi * (k + 0.5) / np);
        D.c_exact(0.5 * t, &vals[size_t(k) * W]);
    }
    std::vector<double> T(size_t(np) * np, 0.0);      // T_q(t) in monomials
    T[0] = 1.0;
    if (np > 1) T[1 * np + 1] = 1.0;
    for (int q = 2; q < np; ++q)
        for (int e = 0; e < np; ++e) {
            double v = -T[(q - 2) * np + e];
            if (e > 0) v += 2.0 * T[(q - 1) * np + e - 1];
            T[q * np + e] = v;
        }
    for (int a = 0; a < W; ++a) {
        std::vector<double> cheb(np, 0.0);
        for (int q = 0; q < np; ++q) {
            double acc = 0;
            for (int k = 0; k < np; ++k) acc += vals[size_t(k) * W + a] * std::cos(kPi * q * (k + 0.5) / np);
            cheb[q] = acc * (q == 0 ? 1.0 : 2.0) / np;
        }
        for (int e = 0; e < np; ++e) {
            double acc = 0;
            for (int q = e; q < np; ++q) acc += cheb[q] * T[q * np + e];
            out[size_t(a) * np + e] = acc * std::ldexp(1.0, e);   // t^e = (2 nu)^e
        }
    }
    return out;
}

}  // namespace

void KernelDesign::c_exact(double nu, double* c) const {
    int nx = int(xn.size());
    std::vector<double> M(A), rhs(W);
    for (int a = 0; a < W; ++a) {
        double acc = 0;
        for (int i = 0; i < nx; ++i)
            acc += std::cos(2.0 * kPi * ((a - 0.5 * (W - 1)) - nu) * xn[i]) * h[i] * wx[i];
        rhs[a] = acc;
    }
    ldlt_solve(W, M, rhs.data(), 1);
    for (int a = 0; a < W; ++a) c[a] = rhs[a];
}

double KernelDesign::c_poly(int a, double nu) const {
    const double* p = &poly[size_t(a) * (degree + 1)];
    double v = p[degree];
    for (int k = degree - 1; k >= 0; --k) v = v * nu + p[k];
    return v;
}

double KernelDesign::c_poly_lo(int a, double nu) const {
    const double* p = &poly_lo[size_t(a) * (degree_lo + 1)];
    double v = p[degree_lo];
    for (int k = degree_lo - 1; k >= 0; --k) v = v * nu + p[k];
    return v;
}

double KernelDesign::h_at(double x) const {
    double num = 0, den = 0;
    int nn = int(nun.size());
    for (int j = 0; j < nn; ++j) {
        double gr = 0, gi = 0;
        for (int a = 0; a < W; ++a) {
            double ang = 2.0 * kPi * ((a - 0.5 * (W - 1)) - nun[j]) * x;
            gr += c_nodes[j * W + a] * std::cos(ang);
            gi += c_nodes[j * W + a] * std::sin(ang);
        }
        num += wn[j] * gr;
        den += wn[j] * (gr * gr + gi * gi);
    }
    return num / den;
}

KernelDesign design_kernel(int W, double x0) {
    if (W < 1 || W > 16) throw std::runtime_error("W must be in [1, 16]");
    if (!(x0 > 0.0 && x0 <= 0.5)) throw std::runtime_error("x0 must be in (0, 1/2]");
    Problem P(W, x0);
    const int nx = P.nx, nn = P.nn;

    // Kaiser-Bessel start: C(u) = I0(beta sqrt(1 - (2u/W)^2)), h pointwise optimal.
    std::vector<double> h, best_h;
    double best_f = -1;
    for (int ib = 0; ib < 400; ++ib) {
        double beta = 0.5 + (3.5 * W - 0.5) * ib / 399.0;
        std::vector<double> c(size_t(nn) * W);
        for (int j = 0; j < nn; ++j)
            for (int a = 0; a < W; ++a) {
                double u = P.s[a] - P.nun[j];
                double t = 1.0 - (2.0 * u / W) * (2.0 * u / W);
                c[j * W + a] = bessel_i0(beta * std::sqrt(std::max(t, 0.0)));
            }
        P.h_from_c(c, h);
        double h0 = h[0];
        for (double& e : h) e /= h0;
        double f = P.sumsq(h);
        if (best_f < 0 || f < best_f) {
            best_f = f;
            best_h = h;
        }
    }
    h = best_h;

    // Levenberg-Marquardt on h[1..nx-1] (h[0] held at its start value).
    const int m = 2 * nn * nx, n = nx - 1;
    std::vector<double> r(m);
    P.residuals(h.data(), r.data());
    double f = 0;
    for (double v : r) f += v * v;
    double lam = 1e-6;
    int iters = 0;
    std::vector<std::complex<double>> hc(nx), rc(m);
    std::vector<double> J(size_t(m) * n), scale(n);
    for (int it = 0; it < 200; ++it) {
        const double step = 1e-40;
        for (int col = 0; col < n; ++col) {
            for (int i = 0; i < nx; ++i) hc[i] = h[i];
            hc[col + 1] += std::complex<double>(0.0, step);
            P.residuals(hc.data(), rc.data());
            double nrm = 0;
            for (int i = 0; i < m; ++i) {
                double v = rc[i].imag() / step;
                J[size_t(col) * m + i] = v;
                nrm += v * v;
            }
            scale[col] = std::sqrt(nrm) > 0 ? std::sqrt(nrm) : 1.0;
            for (int i = 0; i < m; ++i) J[size_t(col) * m + i] /= scale[col];
        }
        bool accepted = false;
        double dmax = 0;
        for (int tries = 0; tries < 80; ++tries) {
            std::vector<double> d = damped_lstsq(J, r, m, n, lam);
            std::vector<double> ht(h);
            dmax = 0;
            for (int k = 0; k < n; ++k) {
                ht[k + 1] += d[k] / scale[k];
                dmax = std::max(dmax, std::fabs(d[k] / scale[k]));
            }
            std::vector<double> rt(m);
            P.residuals(ht.data(), rt.data());
            double ft = 0;
            for (double v : rt) ft += v * v;
            if (ft < f) {
                h.swap(ht);
                r.swap(rt);
                f = ft;
                lam = std::max(lam / 10.0, 1e-24);
                accepted = true;
                break;
            }
            lam *= 4.0;
        }
        iters = it + 1;
        double hmax = *std::max_element(h.begin(), h.end());
        if (!accepted || dmax <= 1e-15 * hmax) break;
    }

    KernelDesign D;
    D.W = W;
    D.x0 = x0;
    D.xn = P.xn;
    D.wx = P.wx;
    D.nun = P.nun;
    D.wn = P.wn;
    D.iterations = iters;
    auto finish = [&](std::vector<double> hv) {
        D.h = std::move(hv);
        D.A.assign(size_t(W) * W, 0.0);
        for (int a = 0; a < W; ++a)
            for (int b = 0; b < W; ++b) {
                double acc = 0;
                for (int i = 0; i < nx; ++i) acc += P.K[(size_t(a) * W + b) * nx + i] * D.h[i] * D.h[i] * D.wx[i];
                D.A[a * W + b] = acc;
            }
        D.c_nodes.assign(size_t(nn) * W, 0.0);
        for (int j = 0; j < nn; ++j) D.c_exact(D.nun[j], &D.c_nodes[size_t(j) * W]);
    };
    finish(h);
    // Scale convention h(0) = 1; C scales inversely and the product is unchanged.
    double h0 = D.h_at(0.0);
    for (double& e : h) e /= h0;
    finish(h);

    D.degree = kDegree;
    D.poly = fit_segments(D, kDegree);
    D.degree_lo = kDegreeLo;
    D.poly_lo = fit_segments(D, kDegreeLo);

    // E on a finer grid, from the fitted polynomials and the pointwise h.
    std::vector<double> fx, fwx, fn, fwn;
    gauss_legendre(120, 0.0, x0, fx, fwx);
    gauss_legendre(120, -0.5, 0.5, fn, fwn);
    std::vector<double> hf(fx.size());
    for (size_t i = 0; i < fx.size(); ++i) hf[i] = D.h_at(fx[i]);
    double e2 = 0;
    for (size_t j = 0; j < fn.size(); ++j) {
        std::vector<double> cv(W);
        for (int a = 0; a < W; ++a) cv[a] = D.c_poly(a, fn[j]);
        for (size_t i = 0; i < fx.size(); ++i) {
            double gr = 0, gi = 0;
            for (int a = 0; a < W; ++a) {
                double ang = 2.0 * kPi * (P.s[a] - fn[j]) * fx[i];
                gr += cv[a] * std::cos(ang);
                gi += cv[a] * std::sin(ang);
            }
            double lr = 1.0 - hf[i] * gr, li = -hf[i] * gi;
            e2 += fwn[j] * fwx[i] * (lr * lr + li * li);
        }
    }
    D.E = std::sqrt(e2 / x0);
    return D;
}

KernelDesign top_hat_design() {
    KernelDesign D;
    D.W = 1;
    D.x0 = 0.5;
    D.degree = kDegree;
    D.poly.assign(size_t(kDegree) + 1, 0.0);
    D.poly[0] = 1.0;
    D.degree_lo = kDegreeLo;
    D.poly_lo.assign(size_t(kDegreeLo) + 1, 0.0);
    D.poly_lo[0] = 1.0;
    D.E = std::nan("");
    return D;
}

std::string make_plan_params_ext(int N, double L, int W, double x0, int Wz, double z0, double wmax, int method,
                                 int n_bins, PlanParams* p) {
    if (N <= 0 || (N & 1)) return "N must be positive and even";
    if (!(x0 > 0.0 && x0 <= 0.5)) return "x0 must be in (0, 1/2]";
    if (W < 1 || W > 16) return "W must be in [1, 16]";
    if (!(L > 0.0 && L < std::sqrt(2.0))) return "L must be in (0, sqrt 2)";
    if (!(wmax >= 0.0) || !std::isfinite(wmax)) return "wmax must be finite and >= 0";
    if (method != kImproved && method != kImprovedNoOffset && method != kOriginal) return "unknown w-layer method";
    if (method == kOriginal) {
        if (Wz != 1) return "the original W-stacking takes W_z = 1 (nearest w bin)";
        if (!(wmax > 0.0)) return "the original W-stacking needs wmax > 0";
        if (n_bins < 0 || n_bins > 1000000) return "n_bins must be in [0, 10^6]";
    } else {
        if (Wz < 1 || Wz > W) return "W_z must be in [1, W]";
        if (!(z0 > 0.0 && z0 <= 0.5)) return "z0 must be in (0, 1/2]";
    }
    double np = N / (2.0 * x0);
    long npr = std::lround(np);
    if (std::fabs(np - double(npr)) > 1e-9) return "N / (2 x0) must be an integer";
    p->N = N;
    p->L = L;
    p->W = W;
    p->Wz = Wz;
    p->x0 = x0;
    p->z0 = method == kOriginal ? 0.0 : z0;
    p->wmax = wmax;
    p->method = method;
    p->Nprime = int(npr);
    p->l_max = 0.5 * L;
    p->n_min = std::sqrt(1.0 - 2.0 * p->l_max * p->l_max);
    p->z_offset = method == kImproved;
    p->w_shift = 0.0;
    p->t_phase = 0.0;
    if (method == kOriginal) {
        // eq. N_w: the smallest integer >= 2 pi (n_max - n_min)(w_max - w_min), w_min = 0 after the fold
        if (n_bins == 0) n_bins = std::max(1, int(std::ceil(2.0 * kPi * (1.0 - p->n_min) * wmax)));
        p->n_bins = n_bins;
        p->n_scale = double(n_bins) / wmax;
        p->n0 = 1.0;
        p->z_shift = 0.0;
        p->w_shift = -0.5;
        p->t_phase = 0.5;
        p->t_lo = 0;
        p->t_hi = n_bins - 1;
        return std::string();
    }
    p->n_bins = 0;
    if (method == kImproved) {
        p->n_scale = (1.0 - p->n_min) / (2.0 * z0);     // eq. n_params
        p->n0 = 1.0 - z0 * p->n_scale;
        p->z_shift = z0;
    } else {
        p->n_scale = (1.0 - p->n_min) / z0;             // eq. n_params_no_offset
        p->n0 = 1.0;
        p->z_shift = 0.0;
    }
    p->t_lo = Wz / 2 - Wz + 1;
    double top = std::floor(p->n_scale * wmax + 0.5 * Wz);
    if (top > 1e6) return "wmax too large: more than a million w-layers";
    p->t_hi = int(top);
    return std::string();
}

std::string make_plan_params(int N, double L, int W, double x0, double wmax, PlanParams* p, bool z_offset) {
    return make_plan_params_ext(N, L, W, x0, W, x0, wmax, z_offset ? kImproved : kImprovedNoOffset, 0, p);
}

}  // namespace wsg
