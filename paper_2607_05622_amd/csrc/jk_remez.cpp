// Remez exchange for the best uniform approximation of 1/x on [1, R] by
// sum_k w_k exp(-t_k x) (see jk_remez.h).
#include "jk_remez.h"

#include <algorithm>
#include <cmath>

namespace jk {
namespace {

struct Sum {
    std::vector<double> lt, lw;   // log t_k, log w_k
    int n() const { return static_cast<int>(lt.size()); }
    double err(double x) const {
        double s = 0.0;
        for (int k = 0; k < n(); ++k) s += std::exp(lw[k] - std::exp(lt[k]) * x);
        return 1.0 / x - s;
    }
    double derr(double x) const {   // d/dx
        double s = 0.0;
        for (int k = 0; k < n(); ++k) {
            const double t = std::exp(lt[k]);
            s += t * std::exp(lw[k] - t * x);
        }
        return -1.0 / (x * x) + s;
    }
};

// Solves the dense system A y = b (A row-major m x m) by elimination with
// partial pivoting.  Returns false when singular.
bool solve(std::vector<double> A, std::vector<double> b, int m, std::vector<double>& y) {
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(A[r * m + c]) > std::fabs(A[p * m + c])) p = r;
        if (!(std::fabs(A[p * m + c]) > 0.0)) return false;
        if (p != c) {
            for (int k = 0; k < m; ++k) std::swap(A[c * m + k], A[p * m + k]);
            std::swap(b[c], b[p]);
        }
        for (int r = c + 1; r < m; ++r) {
            const double f = A[r * m + c] / A[c * m + c];
            if (f == 0.0) continue;
            for (int k = c; k < m; ++k) A[r * m + k] -= f * A[c * m + k];
            b[r] -= f * b[c];
        }
    }
    y.assign(m, 0.0);
    for (int r = m - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < m; ++k) s -= A[r * m + k] * y[k];
        y[r] = s / A[r * m + r];
    }
    for (double v : y)
        if (!std::isfinite(v)) return false;
    return true;
}

// Log-spaced sample of [1, R].
std::vector<double> sample(double R, int m) {
    std::vector<double> x(m);
    const double lr = std::log(R);
    for (int j = 0; j < m; ++j) x[j] = std::exp(lr * j / (m - 1));
    x[0] = 1.0;
    x[m - 1] = R;
    return x;
}

// Weights for fixed nodes: least squares of the error over a log-spaced
// sample (normal equations with a tiny ridge), floored at a small positive
// value so their logarithms exist.
void fit_weights(Sum& s, double R) {
    const int n = s.n();
    const std::vector<double> x = sample(R, 60 * n + 60);
    std::vector<double> A(n * n, 0.0), b(n, 0.0), w;
    for (double xi : x) {
        std::vector<double> e(n);
        for (int k = 0; k < n; ++k) e[k] = std::exp(-std::exp(s.lt[k]) * xi);
        for (int i = 0; i < n; ++i) {
            b[i] += e[i] / xi;
            for (int j = 0; j < n; ++j) A[i * n + j] += e[i] * e[j];
        }
    }
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += A[i * n + i];
    for (int i = 0; i < n; ++i) A[i * n + i] += 1e-14 * tr / n;
    if (!solve(A, b, n, w)) return;
    for (int k = 0; k < n; ++k) s.lw[k] = std::log(std::max(w[k], 1e-12));
}

// Damped Gauss-Newton (Levenberg-Marquardt) on the squared error over a
// log-spaced sample, in log-nodes and log-weights (steps clipped to 1).
void refine_ls(Sum& s, double R) {
    const int n = s.n(), m = 2 * n;
    const std::vector<double> x = sample(R, 40 * n + 40);
    auto cost = [&](const Sum& q) {
        double c = 0.0;
        for (double xi : x) {
            const double e = q.err(xi) * xi;
            c += e * e;
        }
        return c;
    };
    double c0 = cost(s), lambda = 1e-3;
    for (int it = 0; it < 200; ++it) {
        std::vector<double> JtJ(m * m, 0.0), Jtr(m, 0.0), g(m);
        for (double xi : x) {
            const double r = s.err(xi) * xi;
            for (int k = 0; k < n; ++k) {
                const double t = std::exp(s.lt[k]), e = std::exp(s.lw[k] - t * xi);
                g[k] = e * t * xi * xi;
                g[n + k] = -e * xi;
            }
            for (int i = 0; i < m; ++i) {
                Jtr[i] += g[i] * r;
                for (int j = 0; j < m; ++j) JtJ[i * m + j] += g[i] * g[j];
            }
        }
        bool accepted = false;
        for (int tries = 0; tries < 16 && !accepted; ++tries) {
            std::vector<double> A = JtJ, b(m), d;
            for (int i = 0; i < m; ++i) {
                A[i * m + i] = A[i * m + i] * (1.0 + lambda) + 1e-300;
                b[i] = -Jtr[i];
            }
            if (!solve(A, b, m, d)) {
                lambda *= 10.0;
                continue;
            }
            Sum q = s;
            for (int k = 0; k < n; ++k) {
                q.lt[k] += std::max(-2.0, std::min(2.0, d[k]));
                q.lw[k] += std::max(-2.0, std::min(2.0, d[n + k]));
            }
            const double c1 = cost(q);
            if (c1 < c0) {
                const bool stalled = c0 - c1 <= 1e-14 * c0;
                s = q;
                c0 = c1;
                lambda = std::max(lambda * 0.3, 1e-12);
                if (stalled) return;
                accepted = true;
            } else {
                lambda *= 10.0;
            }
        }
        if (!accepted) return;
    }
}

// Start from scratch: the trapezoid rule in u = log t for 1/x = int exp(u -
// x e^u) du over a range covering x in [1, R], refined by least squares.
Sum sinc_start(int n, double R) {
    Sum s;
    const double a = -std::log(R) - 3.0 - 0.3 * std::sqrt(static_cast<double>(n)),
                 b = 1.5 + 0.3 * std::sqrt(static_cast<double>(n));
    const double h = n > 1 ? (b - a) / (n - 1) : 1.0;
    for (int k = 0; k < n; ++k) {
        const double u = n > 1 ? a + h * k : 0.5 * (a + b) - 0.5 * std::log(R);
        s.lt.push_back(u);
        s.lw.push_back(u + std::log(h));
    }
    refine_ls(s, R);
    return s;
}

// Start for k + 1 terms from the best k-term sum, by one of several rules
// (tried in turn): the old terms kept and a new one of negligible weight put
// above the old top or below the old bottom node (the error curve is then
// still the old alternant); or the old nodes moved down by delta in log t
// and the new one put on top with a guessed weight.  One term: a node near
// the middle of log [1/R, 1], weight refitted.
constexpr int kGrowRules = 10;
Sum grow(const Sum& prev, double R, int rule) {
    Sum s;
    const int k = prev.n();
    if (k == 0) {
        s.lt.push_back(-0.5 * std::log(R) - 0.5);
        s.lw.push_back(0.0);
        fit_weights(s, R);
        return s;
    }
    std::vector<int> o(k);
    for (int i = 0; i < k; ++i) o[i] = i;
    std::sort(o.begin(), o.end(), [&](int a, int b) { return prev.lt[a] < prev.lt[b]; });
    const double top = prev.lt[o[k - 1]], bot = prev.lt[o[0]];
    const double gtop = k > 1 ? top - prev.lt[o[k - 2]] : 1.0, gbot = k > 1 ? prev.lt[o[1]] - bot : 1.0;
    static const double deltas[kGrowRules - 2] = {1.0, 0.8, 1.2, 0.6, 1.4, 0.4, 0.2, 0.0};
    const double delta = rule >= 2 ? deltas[rule - 2] : 0.0;
    for (int i : o) {
        s.lt.push_back(prev.lt[i] - delta);
        s.lw.push_back(prev.lw[i] - delta);
    }
    // the new term's weight for rules 0 and 1: its size at the end of [1, R]
    // it acts on is the current error level E
    const double lE = std::log(std::max(std::fabs(prev.err(1.0)), 1e-300));
    if (rule == 0) {
        const double lt = top + gtop;
        s.lt.push_back(lt);
        s.lw.push_back(lE + std::exp(lt));
    } else if (rule == 1) {
        const double lt = bot - gbot;
        s.lt.insert(s.lt.begin(), lt);
        s.lw.insert(s.lw.begin(), lE + std::exp(lt) * R);
    } else {
        const double off = prev.lw[o[k - 1]] - top;
        s.lt.push_back(top + 0.8 * gtop);
        s.lw.push_back(top + 0.8 * gtop + 0.6 * off);
    }
    return s;
}

// Extrema of the error curve: both ends and the interior zeros of its
// derivative, bracketed on a dense log grid and refined by bisection.
std::vector<double> extrema(const Sum& s, double R) {
    const std::vector<double> x = sample(R, 400 * s.n() + 400);
    std::vector<double> ext{1.0};
    double d0 = s.derr(x[0]);
    for (size_t j = 1; j < x.size(); ++j) {
        const double d1 = s.derr(x[j]);
        if ((d0 < 0.0) != (d1 < 0.0) && j + 1 < x.size()) {
            double lo = x[j - 1], hi = x[j], dlo = d0;
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + hi), dm = s.derr(mid);
                if ((dm < 0.0) == (dlo < 0.0)) {
                    lo = mid;
                    dlo = dm;
                } else {
                    hi = mid;
                }
                if (hi - lo <= 1e-15 * hi) break;
            }
            ext.push_back(0.5 * (lo + hi));
        }
        d0 = d1;
    }
    ext.push_back(R);
    // alternate in sign: of neighbours with one sign keep the larger
    std::vector<double> alt;
    for (double e : ext) {
        if (!alt.empty() && (s.err(alt.back()) < 0.0) == (s.err(e) < 0.0)) {
            if (std::fabs(s.err(e)) > std::fabs(s.err(alt.back()))) alt.back() = e;
        } else {
            alt.push_back(e);
        }
    }
    return alt;
}


// Remez exchange from the start s; true when the extrema level out.
bool exchange(Sum& s, double R, int& iters, const std::vector<double>* ref0 = nullptr) {
    const int n = s.n(), m = 2 * n + 1;
    double E = 0.0;
    int short_refs = 0;
    for (int outer = 0; outer < 100; ++outer) {
        iters = outer;
        std::vector<double> ext = extrema(s, R);
        // a given first reference (2n + 1 points) replaces a short alternant
        if (outer == 0 && ref0 && static_cast<int>(ref0->size()) == m && static_cast<int>(ext.size()) < m) ext = *ref0;
        // more alternation points than needed: drop the smaller end
        while (static_cast<int>(ext.size()) > m) {
            if (std::fabs(s.err(ext.front())) < std::fabs(s.err(ext.back()))) ext.erase(ext.begin());
            else ext.pop_back();
        }
        const bool madeup = static_cast<int>(ext.size()) < m;
        if (madeup && ++short_refs > 20) return false;   // no alternant in sight
        if (madeup) {
            // too few: a reference set made up to 2n + 1 points by splitting the
            // widest gaps (in log x); Newton then imposes the alternation on it
            while (static_cast<int>(ext.size()) < m) {
                size_t g = 0;
                double best = -1.0;
                for (size_t i = 0; i + 1 < ext.size(); ++i) {
                    const double r = ext[i + 1] / ext[i];
                    if (r > best) {
                        best = r;
                        g = i;
                    }
                }
                ext.insert(ext.begin() + g + 1, std::sqrt(ext[g] * ext[g + 1]));
            }
        }
        double emax = 0.0, emin = 1e300;
        for (double e : ext) {
            emax = std::max(emax, std::fabs(s.err(e)));
            emin = std::min(emin, std::fabs(s.err(e)));
        }
        // level to 1e-7 on the curve's own extrema, or to the rounding floor
        // of the error sums (terms of order one)
        if (!madeup && emax - emin <= std::max(1e-7 * emax, 2e-14)) return true;
        // Newton on err(x_i) - (-1)^i E = 0 with the points fixed
        const double sg = s.err(ext[0]) > 0.0 ? 1.0 : -1.0;
        E = sg * 0.5 * (emax + emin);
        for (int it = 0; it < 60; ++it) {
            std::vector<double> A(m * m), F(m);
            double f0 = 0.0;
            for (int i = 0; i < m; ++i) {
                const double xi = ext[i], si = (i % 2) ? -1.0 : 1.0;
                F[i] = s.err(xi) - si * E;
                f0 += F[i] * F[i];
                for (int k = 0; k < n; ++k) {
                    const double t = std::exp(s.lt[k]), e = std::exp(s.lw[k] - t * xi);
                    A[i * m + k] = e * t * xi;   // d err / d log t_k
                    A[i * m + n + k] = -e;       // d err / d log w_k
                }
                A[i * m + 2 * n] = -si;
            }
            std::vector<double> b(m), d;
            for (int i = 0; i < m; ++i) b[i] = -F[i];
            if (!solve(A, b, m, d)) return false;
            // steps of at most 1 in the logarithms
            double step = 1.0, maxd = 0.0;
            for (int k = 0; k < 2 * n; ++k) maxd = std::max(maxd, std::fabs(d[k]));
            if (maxd > 1.0) step = 1.0 / maxd;
            bool moved = false;
            for (int tries = 0; tries < 30; ++tries) {
                Sum q = s;
                for (int k = 0; k < n; ++k) {
                    q.lt[k] += step * d[k];
                    q.lw[k] += step * d[n + k];
                }
                const double Eq = E + step * d[2 * n];
                double f1 = 0.0;
                for (int i = 0; i < m; ++i) {
                    const double fi = q.err(ext[i]) - ((i % 2) ? -1.0 : 1.0) * Eq;
                    f1 += fi * fi;
                }
                if (f1 < f0 || f1 == 0.0) {
                    s = q;
                    E = Eq;
                    moved = true;
                    break;
                }
                step *= 0.5;
            }
            if (!moved || maxd * step < 1e-14) break;
        }
    }
    return false;
}


// The best n-term sum on [1, R] by continuation in the number of terms
// (each from the last); false if a step fails.
bool grow_to(int n, double R, Sum& s, int& iters, bool& floor) {
    s = Sum();
    floor = false;
    for (int k = 1; k <= n; ++k) {
        bool ok = false;
        for (int c = 0; c <= kGrowRules && !ok; ++c) {
            Sum q = (c < kGrowRules && k > 1) ? grow(s, R, c) : sinc_start(k, R);
            int it = 0;
            if (exchange(q, R, it)) {
                s = q;
                ok = true;
            }
            iters += it;
            if (k == 1) c = kGrowRules;
        }
        if (!ok) return false;
        // below 1e-12 the error curve is rounding noise: more terms cannot be placed
        if (k < n && std::fabs(s.err(1.0)) < 1e-12) {
            floor = true;
            return false;
        }
    }
    return true;
}

}  // namespace

RemezResult remez_inverse(int n, double R) {
    RemezResult res;
    if (n < 1 || !(R > 1.0) || !std::isfinite(R)) return res;
    Sum s;
    bool floor = false;
    res.ok = grow_to(n, R, s, res.iterations, floor);
    res.precision_limited = floor;
    if (!res.ok && !floor) {
        // continuation in the interval: solve on a longer [1, R'] (better
        // conditioned for many terms) and shrink R' to R in small steps, each
        // exchange starting from the last solution
        for (double Rs = R * 10.0; Rs <= R * 1000.0 && !res.ok; Rs *= 10.0) {
            if (!grow_to(n, Rs, s, res.iterations, floor)) continue;
            bool ok = true;
            for (double r = Rs; r > R && ok;) {
                // the last alternant, compressed in log x into the shorter interval
                std::vector<double> ref = extrema(s, r);
                const double rn = std::max(R, r * 0.8);
                for (double& x : ref) x = std::exp(std::log(x) * std::log(rn) / std::log(r));
                r = rn;
                int it = 0;
                ok = exchange(s, r, it, &ref);
                res.iterations += it;
            }
            res.ok = ok;
        }
    }
    std::vector<int> order(s.n());
    for (int k = 0; k < s.n(); ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return s.lt[a] < s.lt[b]; });
    for (int k : order) {
        res.t.push_back(std::exp(s.lt[k]));
        res.w.push_back(std::exp(s.lw[k]));
    }
    double e = 0.0;
    if (s.n() > 0) {
        for (double x : sample(R, 2000 * s.n() + 2000)) e = std::max(e, std::fabs(s.err(x)));
        for (double x : extrema(s, R)) e = std::max(e, std::fabs(s.err(x)));
    }
    res.err = e;
    return res;
}

}  // namespace jk
