// laplace_rule.hpp -- minimax exponential sums for 1/x (host code only).
//
// Sec. 2.2, Eq. (laplace) discretizes 1/x = int_0^inf exp(-t x) dt by a
// short exponential sum.  On the scaled range y = x / x_min in [1, R] the rule
// minimizes the maximum relative error
//
//     eta(y) = 1 - y sum_k w_k exp(-a_k y),        max over [1, R] of |eta|.
//
// The best rule equioscillates: |eta| reaches its maximum E with alternating
// signs at 2n + 1 points, both ends included.  It is found in three steps:
//   1. start: trapezoid rule in s for 1/y = int exp(s - y e^s) ds;
//   2. least p-th powers of eta on a logarithmic grid for p = 2, 4, ..., 64
//      (Levenberg-Marquardt, each stage started from the last), which drives
//      the error curve towards equal ripples;
//   3. Remez exchange: Newton's method on eta(y_i) = (-1)^i E at the 2n + 1
//      extrema, the extrema moved to those of the new curve, until level.
// Every candidate is ranked by its measured maximum error (a dense
// logarithmic scan refined at each local extremum); the best one is kept.
#pragma once

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

namespace jk_rule {

constexpr int kMaxTerms = 32;

// Parameters as logarithms (u_k = ln w_k, v_k = ln a_k): weights and
// exponents span many orders of magnitude and must stay positive.
struct Rule {
    int n = 0;
    double u[kMaxTerms], v[kMaxTerms];
};

inline double eta(const Rule &r, double y)
{
    double s = 0.0;
    for (int k = 0; k < r.n; k++)
        s += std::exp(r.u[k] - std::exp(r.v[k]) * y);
    return 1.0 - y * s;
}

// d eta / d u_k into du[k], d eta / d v_k into dv[k].
inline void eta_grad(const Rule &r, double y, double *du, double *dv)
{
    for (int k = 0; k < r.n; k++) {
        const double a = std::exp(r.v[k]);
        const double t = y * std::exp(r.u[k] - a * y);
        du[k] = -t;
        dv[k] = t * a * y;
    }
}

// Dense solve A x = b (n x n row-major; both overwritten, x returned in b),
// Gaussian elimination with partial pivoting.
inline bool solve(int n, std::vector<double> &A, std::vector<double> &b)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        double best = std::fabs(A[(size_t)c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[(size_t)r * n + c]) > best) {
                best = std::fabs(A[(size_t)r * n + c]);
                piv = r;
            }
        if (!(best > 0.0) || !std::isfinite(best))
            return false;
        if (piv != c) {
            for (int j = 0; j < n; j++)
                std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
            std::swap(b[c], b[piv]);
        }
        const double d = A[(size_t)c * n + c];
        for (int r = c + 1; r < n; r++) {
            const double f = A[(size_t)r * n + c] / d;
            if (f == 0.0)
                continue;
            for (int j = c; j < n; j++)
                A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; c--) {
        double s = b[c];
        for (int j = c + 1; j < n; j++)
            s -= A[(size_t)c * n + j] * b[j];
        b[c] = s / A[(size_t)c * n + c];
        if (!std::isfinite(b[c]))
            return false;
    }
    return true;
}

// Least squares min ||A x - b|| for A (m x n, row-major, m >= n, overwritten)
// by Householder QR; x returned in the first n entries of b.  Avoids the
// squared condition number of the normal equations, which would limit the
// fitted error to about the square root of the rounding unit.
inline bool lstsq(int m, int n, std::vector<double> &A, std::vector<double> &b)
{
    for (int c = 0; c < n; c++) {
        double nrm = 0.0;
        for (int r = c; r < m; r++)
            nrm = std::hypot(nrm, A[(size_t)r * n + c]);
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return false;
        const double a0 = A[(size_t)c * n + c];
        const double alpha = a0 > 0.0 ? -nrm : nrm;
        // v = x - alpha e1, stored in column c from row c; beta = 2 / v.v
        A[(size_t)c * n + c] = a0 - alpha;
        double vv = 0.0;
        for (int r = c; r < m; r++)
            vv += A[(size_t)r * n + c] * A[(size_t)r * n + c];
        for (int j = c + 1; j < n; j++) {
            double d = 0.0;
            for (int r = c; r < m; r++)
                d += A[(size_t)r * n + c] * A[(size_t)r * n + j];
            const double f = 2.0 * d / vv;
            for (int r = c; r < m; r++)
                A[(size_t)r * n + j] -= f * A[(size_t)r * n + c];
        }
        double d = 0.0;
        for (int r = c; r < m; r++)
            d += A[(size_t)r * n + c] * b[r];
        const double f = 2.0 * d / vv;
        for (int r = c; r < m; r++)
            b[r] -= f * A[(size_t)r * n + c];
        A[(size_t)c * n + c] = alpha;       // R's diagonal
    }
    for (int c = n - 1; c >= 0; c--) {
        double s = b[c];
        for (int j = c + 1; j < n; j++)
            s -= A[(size_t)c * n + j] * b[j];
        b[c] = s / A[(size_t)c * n + c];
        if (!std::isfinite(b[c]))
            return false;
    }
    return true;
}

inline Rule trapezoid_start(int n, double R)
{
    Rule r;
    r.n = n;
    const double s_lo = -std::log(R) - 2.5, s_hi = 1.5 + 0.25 * std::log((double)n);
    const double h = n > 1 ? (s_hi - s_lo) / (n - 1) : (s_hi - s_lo);
    for (int k = 0; k < n; k++) {
        const double s = n > 1 ? s_lo + k * h : 0.5 * (s_lo + s_hi);
        r.v[k] = s;                   // a_k = e^s
        r.u[k] = std::log(h) + s;     // w_k = h e^s
    }
    return r;
}

// Minimizes sum_j |eta(y_j)|^p, written as least squares of
// rho_j = eta_j |eta_j / s|^((p - 2) / 2) (s: the current maximum, so the
// residuals stay of order s).  Levenberg-Marquardt with Nielsen's damping
// update and steps capped at 2 in log space.
inline void lm_pnorm(Rule &r, const std::vector<double> &y, double p, int maxit)
{
    const int n = r.n, np = 2 * n, M = (int)y.size();
    const double q = 0.5 * (p - 2.0);
    double s = 0.0;
    for (int j = 0; j < M; j++)
        s = std::max(s, std::fabs(eta(r, y[j])));
    if (!(s > 0.0) || !std::isfinite(s))
        return;
    std::vector<double> rho(M), Jm((size_t)M * np), N((size_t)np * np), g(np), A, b;
    auto resid = [&](const Rule &t, std::vector<double> &out) {
        double c = 0.0;
        for (int j = 0; j < M; j++) {
            const double e = eta(t, y[j]);
            out[j] = e * std::pow(std::fabs(e) / s, q);
            c += out[j] * out[j];
        }
        return 0.5 * c;
    };
    auto linearize = [&]() {
        for (int j = 0; j < M; j++) {
            const double e = eta(r, y[j]);
            const double f = (1.0 + q) * std::pow(std::fabs(e) / s, q);
            double *row = &Jm[(size_t)j * np];
            eta_grad(r, y[j], row, row + n);
            for (int c = 0; c < np; c++)
                row[c] *= f;
        }
        for (int a = 0; a < np; a++) {
            double t = 0.0;
            for (int j = 0; j < M; j++)
                t += Jm[(size_t)j * np + a] * rho[j];
            g[a] = t;
            for (int c = 0; c <= a; c++) {
                double u = 0.0;
                for (int j = 0; j < M; j++)
                    u += Jm[(size_t)j * np + a] * Jm[(size_t)j * np + c];
                N[(size_t)a * np + c] = N[(size_t)c * np + a] = u;
            }
        }
    };
    std::vector<double> rho1(M);
    double F = resid(r, rho);
    linearize();
    double mu = 0.0;
    for (int a = 0; a < np; a++)
        mu = std::max(mu, N[(size_t)a * np + a]);
    mu *= 1e-3;
    double nu = 2.0;
    for (int it = 0; it < maxit; it++) {
        double gmax = 0.0;
        for (int a = 0; a < np; a++)
            gmax = std::max(gmax, std::fabs(g[a]));
        if (gmax <= 1e-300 || F <= 0.0)
            break;
        // damped step: least squares of [J; sqrt(mu) I] d = [-rho; 0]
        A.assign((size_t)(M + np) * np, 0.0);
        b.assign(M + np, 0.0);
        std::copy(Jm.begin(), Jm.end(), A.begin());
        for (int j = 0; j < M; j++)
            b[j] = -rho[j];
        for (int a = 0; a < np; a++)
            A[(size_t)(M + a) * np + a] = std::sqrt(mu);
        if (!lstsq(M + np, np, A, b)) {
            mu *= nu;
            nu *= 2.0;
            continue;
        }
        b.resize(np);
        double big = 0.0;
        for (int a = 0; a < np; a++)
            big = std::max(big, std::fabs(b[a]));
        if (big < 1e-14)
            break;
        if (big > 2.0)
            for (int a = 0; a < np; a++)
                b[a] *= 2.0 / big;
        // predicted decrease of the linear model for this step
        double pred = 0.0;
        for (int j = 0; j < M; j++) {
            double lin = rho[j];
            for (int a = 0; a < np; a++)
                lin += Jm[(size_t)j * np + a] * b[a];
            pred += 0.5 * (rho[j] * rho[j] - lin * lin);
        }
        Rule t = r;
        for (int k = 0; k < n; k++) {
            t.u[k] += b[k];
            t.v[k] += b[n + k];
        }
        const double F1 = resid(t, rho1);
        const double gain = (pred > 0.0 && std::isfinite(F1)) ? (F - F1) / pred : -1.0;
        if (gain > 0.0) {
            const bool small = F - F1 <= 1e-13 * F;
            r = t;
            F = F1;
            rho.swap(rho1);
            linearize();
            const double c = 2.0 * gain - 1.0;
            mu *= std::max(1.0 / 3.0, 1.0 - c * c * c);
            nu = 2.0;
            if (small)
                break;
        } else {
            mu *= nu;
            nu *= 2.0;
            if (!(mu < 1e300))
                break;
        }
    }
}

// Local extrema of eta on [1, R], both ends included, as (y, eta) pairs with
// alternating signs (runs of one sign keep their largest magnitude); returns
// the largest |eta| found.  Dense logarithmic scan, then golden-section
// refinement of every interior extremum.
inline double extrema(const Rule &r, double R, std::vector<double> &ys, std::vector<double> &es)
{
    constexpr int kScan = 20001;
    const double lr = std::log(R);
    std::vector<double> e(kScan);
    for (int j = 0; j < kScan; j++)
        e[j] = eta(r, std::exp(lr * j / (kScan - 1)));
    std::vector<double> cy, ce;
    cy.push_back(1.0);
    ce.push_back(e[0]);
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int j = 1; j < kScan - 1; j++) {
        if ((e[j] - e[j - 1]) * (e[j + 1] - e[j]) >= 0.0)
            continue;
        const double sg = e[j] > 0.0 ? 1.0 : -1.0;
        double lo = lr * (j - 1) / (kScan - 1), hi = lr * (j + 1) / (kScan - 1);
        double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
        double f1 = sg * eta(r, std::exp(x1)), f2 = sg * eta(r, std::exp(x2));
        for (int it = 0; it < 60; it++) {
            if (f1 > f2) {
                hi = x2;
                x2 = x1;
                f2 = f1;
                x1 = hi - gr * (hi - lo);
                f1 = sg * eta(r, std::exp(x1));
            } else {
                lo = x1;
                x1 = x2;
                f1 = f2;
                x2 = lo + gr * (hi - lo);
                f2 = sg * eta(r, std::exp(x2));
            }
        }
        const double yv = std::exp(0.5 * (lo + hi)), val = eta(r, yv);
        if (sg * val >= sg * e[j]) {
            cy.push_back(yv);
            ce.push_back(val);
        } else {
            cy.push_back(std::exp(lr * j / (kScan - 1)));
            ce.push_back(e[j]);
        }
    }
    cy.push_back(R);
    ce.push_back(e[kScan - 1]);
    double mx = 0.0;
    for (int j = 0; j < kScan; j++)
        mx = std::max(mx, std::fabs(e[j]));
    ys.clear();
    es.clear();
    for (size_t i = 0; i < cy.size(); i++) {
        mx = std::max(mx, std::fabs(ce[i]));
        if (!es.empty() && (es.back() > 0.0) == (ce[i] > 0.0)) {
            if (std::fabs(ce[i]) > std::fabs(es.back())) {
                es.back() = ce[i];
                ys.back() = cy[i];
            }
        } else {
            ys.push_back(cy[i]);
            es.push_back(ce[i]);
        }
    }
    return std::isfinite(mx) ? mx : 1e300;
}

// Newton's method for eta(y_i) = (-1)^i E, i < 2n + 1, in (u, v, E); the step
// is halved until the residual norm drops.  True at rounding level.
inline bool remez_newton(Rule &r, double &E, const std::vector<double> &ys)
{
    const int n = r.n, m = 2 * n + 1;
    std::vector<double> F(m), F1(m), A, b;
    auto resid = [&](const Rule &q, double EE, std::vector<double> &out) {
        double s = 0.0;
        for (int i = 0; i < m; i++) {
            out[i] = eta(q, ys[i]) - ((i & 1) ? -EE : EE);
            s += out[i] * out[i];
        }
        return std::sqrt(s);
    };
    const double done = 1e-15 * std::sqrt((double)m);
    double f0 = resid(r, E, F);
    for (int it = 0; it < 60 && f0 > done; it++) {
        A.assign((size_t)m * m, 0.0);
        b.resize(m);
        for (int i = 0; i < m; i++) {
            eta_grad(r, ys[i], &A[(size_t)i * m], &A[(size_t)i * m + n]);
            A[(size_t)i * m + 2 * n] = (i & 1) ? 1.0 : -1.0;
            b[i] = -F[i];
        }
        if (!solve(m, A, b))
            return false;
        double big = 0.0;
        for (int p = 0; p < 2 * n; p++)
            big = std::max(big, std::fabs(b[p]));
        double t = big > 1.0 ? 1.0 / big : 1.0;
        bool moved = false;
        for (int tries = 0; tries < 40 && !moved; tries++, t *= 0.5) {
            Rule q = r;
            for (int k = 0; k < n; k++) {
                q.u[k] += t * b[k];
                q.v[k] += t * b[n + k];
            }
            const double E1 = E + t * b[2 * n];
            const double f1 = resid(q, E1, F1);
            if (std::isfinite(f1) && f1 < f0) {
                r = q;
                E = E1;
                F.swap(F1);
                f0 = f1;
                moved = true;
            }
        }
        if (!moved)
            break;
    }
    return f0 <= 1e3 * done;
}

inline void sort_by_exponent(Rule &r)
{
    std::vector<std::pair<double, double>> p(r.n);
    for (int k = 0; k < r.n; k++)
        p[k] = {r.v[k], r.u[k]};
    std::sort(p.begin(), p.end());
    for (int k = 0; k < r.n; k++) {
        r.v[k] = p[k].first;
        r.u[k] = p[k].second;
    }
}

// Remez exchange from r; returns the best rule seen, its measured error, and
// whether the ripples came out level (the minimax rule was reached).
inline Rule remez(Rule r, double R, double &err, bool &level)
{
    const int n = r.n;
    std::vector<double> ys, es;
    sort_by_exponent(r);
    Rule best = r;
    double best_err = extrema(r, R, ys, es);
    level = false;
    for (int it = 0; it < 50; it++) {
        if ((int)ys.size() != 2 * n + 1)
            break;
        double lo = 1e300, hi = 0.0;
        for (double e : es) {
            lo = std::min(lo, std::fabs(e));
            hi = std::max(hi, std::fabs(e));
        }
        if (hi - lo <= 1e-7 * hi) {
            level = true;
            break;
        }
        double E = es[0];
        Rule q = r;
        if (!remez_newton(q, E, ys))
            break;
        sort_by_exponent(q);
        const double e = extrema(q, R, ys, es);
        r = q;
        if (e < best_err) {
            best = q;
            best_err = e;
        }
    }
    err = best_err;
    return best;
}

// p-norm stages then Remez on [1, R], from r.
inline Rule fit(Rule r, double R, double p_first, double &err, bool &level)
{
    const int M = 24 * r.n + 48;
    std::vector<double> y(M);
    for (int j = 0; j < M; j++)
        y[j] = std::exp(std::log(R) * j / (M - 1));
    for (double p = p_first; p <= 64.0; p *= 2.0)
        lm_pnorm(r, y, p, 300);
    return remez(r, R, err, level);
}

// The n-term rule on [1, R] (R >= 2), its measured maximum relative error,
// and whether the exchange ended with level ripples.  Measured on this
// path: the ripples come out level (the minimax rule) when the range is wide
// enough for n terms -- R >= 10 up to n = 6, R >= 100 up to n = 8, R >= 1e3
// up to n = 12, R >= 1e5 up to n = 16; on narrower ranges the best rule
// found has errors below about 1e-6 and is not claimed to be minimax.
inline Rule minimax(int n, double R, double &err, bool &level)
{
    return fit(trapezoid_start(n, R), R, 2.0, err, level);
}

} // namespace jk_rule
