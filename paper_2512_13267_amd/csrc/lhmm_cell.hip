// lhmm_cell.hip -- host-side recipe for the initial in-plane lattice of a
// micro-box that must survive a constant in-plane velocity gradient
// (include/lhmm.h, lhmm_box_cell).
//
// A periodic cell deformed by dh/dt = L h (the homogeneous imposition of
// the macro gradient, Eq. micro_bc) stays usable only while its reduced
// lattice keeps every perpendicular width above a few cutoffs.  Three
// shapes are offered, tried in this order:
//   cubic:    kept when its reduced lattice stays at least min_width wide
//             over [0, t_run];
//   rotated:  a rotational or shear-like gradient (a^2 + bc <= 0) stretches
//             a lattice at most linearly in time; the square lattice of side
//             `edge` rotated to the angle whose narrowest width over
//             [0, t_run] is largest;
//   KR:       a hyperbolic gradient (a^2 + bc = k^2 > 0): a lattice aligned
//             in the manner of Kraynik and Reinelt, whose basis P satisfies
//             exp(L T) P = P M with the integer matrix M = [[2, 1], [1, 1]]
//             (eigenvalues mu = (3 + sqrt 5)/2 and 1/mu), so the flow maps
//             the lattice onto itself every period T = ln(mu)/k and the
//             reduced cell's widths are periodic in time.  The family
//             P = V diag(r, +-1) W^-1 (V, W eigenvectors of L and M) scaled
//             to area edge^2 is searched for the member whose narrowest
//             width over one period is largest (the members are time shifts
//             of one another, so near-ties are broken by the width at t = 0).
// The returned basis is the lattice's reduced one (its two successive
// minima, positive orientation); the z extent stays `edge`.  Plain double
// arithmetic without contraction, so the result does not depend on the
// compiler's fusing of products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lhmm.h"
#include "lhmm_internal.h"

#pragma clang fp contract(off)

namespace {

struct M2 {
    double a, b, c, d;  // [[a, b], [c, d]]; columns are lattice vectors
};

M2 mul(const M2& x, const M2& y) {
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}

double det(const M2& x) { return x.a * x.d - x.b * x.c; }

// exp(L t) for traceless L = [[a, b], [c, -a]]: L^2 = k^2 I, so
// exp(L t) = f0 I + f1 L with (cosh, sinh/k), (cos, sin/w) or (1, t)
M2 expm(double a, double b, double c, double t) {
    const double k2 = a * a + b * c;
    double f0, f1;
    if (k2 > 0.0) {
        const double k = std::sqrt(k2);
        f0 = std::cosh(k * t);
        f1 = std::sinh(k * t) / k;
    } else if (k2 < 0.0) {
        const double w = std::sqrt(-k2);
        f0 = std::cos(w * t);
        f1 = std::sin(w * t) / w;
    } else {
        f0 = 1.0;
        f1 = t;
    }
    return {f0 + f1 * a, f1 * b, f1 * c, f0 - f1 * a};
}

// Largest achievable narrowest perpendicular width of the lattice with
// basis B: area / (second successive minimum), the minima found among the
// vectors m b1 + n b2, |m|, |n| <= K.
double lattice_min_width(const M2& B, int K) {
    const double area = std::fabs(det(B));
    double l1 = INFINITY, v1x = 0.0, v1y = 0.0;
    for (int m = -K; m <= K; ++m)
        for (int n = -K; n <= K; ++n) {
            if (m == 0 && n == 0) continue;
            const double x = B.a * m + B.b * n, y = B.c * m + B.d * n;
            const double l = std::hypot(x, y);
            if (l < l1) {
                l1 = l;
                v1x = x;
                v1y = y;
            }
        }
    double l2 = INFINITY;
    for (int m = -K; m <= K; ++m)
        for (int n = -K; n <= K; ++n) {
            if (m == 0 && n == 0) continue;
            const double x = B.a * m + B.b * n, y = B.c * m + B.d * n;
            const double l = std::hypot(x, y);
            if (std::fabs(v1x * y - v1y * x) > 1e-9 * l1 * l && l < l2) l2 = l;
        }
    return area / l2;
}

// narrowest width of the lattice B carried by the flow over n_t equally
// spaced times of [0, t_end]
double min_width_over(double a, double b, double c, const M2& B, double t_end, int n_t, int K) {
    double w = INFINITY;
    for (int i = 0; i < n_t; ++i) {
        const double t = n_t > 1 ? t_end * i / (n_t - 1) : 0.0;
        w = std::min(w, lattice_min_width(mul(expm(a, b, c, t), B), K));
    }
    return w;
}

// The lattice's two successive minima as a positively oriented basis:
// lattice vectors by length (ties in enumeration order), the shortest, then
// the shortest independent of it.
bool short_basis(const M2& B, M2* out) {
    constexpr int K = 12;
    struct V {
        double l, x, y;
        int idx;
    };
    std::vector<V> vs;
    vs.reserve((2 * K + 1) * (2 * K + 1));
    int idx = 0;
    for (int m = -K; m <= K; ++m)
        for (int n = -K; n <= K; ++n) {
            if (m == 0 && n == 0) continue;
            const double x = B.a * m + B.b * n, y = B.c * m + B.d * n;
            vs.push_back({std::hypot(x, y), x, y, idx++});
        }
    std::stable_sort(vs.begin(), vs.end(), [](const V& p, const V& q) { return p.l < q.l; });
    const V& v1 = vs[0];
    for (size_t k = 1; k < vs.size(); ++k) {
        double x = vs[k].x, y = vs[k].y;
        const double cross = v1.x * y - v1.y * x;
        if (std::fabs(cross) > 1e-9 * v1.l * vs[k].l) {
            if (cross < 0) {
                x = -x;
                y = -y;
            }
            *out = {v1.x, x, v1.y, y};
            return std::fabs(std::fabs(det(*out)) - std::fabs(det(B))) <= 1e-9 * std::fabs(det(B));
        }
    }
    return false;
}

// unit eigenvector of [[a, b], [c, -a]] for the eigenvalue lam (real)
void eigvec(double a, double b, double c, double lam, double* x, double* y) {
    // (a - lam) x + b y = 0  or  c x + (-a - lam) y = 0: take the better row
    double u, v;
    if (std::hypot(a - lam, b) >= std::hypot(c, -a - lam)) {
        u = b;
        v = lam - a;
    } else {
        u = lam + a;
        v = c;
    }
    const double n = std::hypot(u, v);
    *x = u / n;
    *y = v / n;
}

}  // namespace

extern "C" int lhmm_box_cell(const double* L, double edge, double t_run, double min_width, double* h_out,
                             int32_t* kind) {
    lhmm_clear_error();
    if (!L || !h_out) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(L[k])) return lhmm_fail(LHMM_ERR_ARG, "gradient not finite");
    if (L[2] != 0.0 || L[5] != 0.0 || L[6] != 0.0 || L[7] != 0.0 || L[8] != 0.0 ||
        std::fabs(L[0] + L[4]) > 1e-12 * (1.0 + std::fabs(L[0]) + std::fabs(L[4])))
        return lhmm_fail(LHMM_ERR_ARG, "the gradient must be in-plane and traceless");
    if (!(edge > 0.0) || !std::isfinite(edge) || !(t_run >= 0.0) || !std::isfinite(t_run) || !(min_width > 0.0))
        return lhmm_fail(LHMM_ERR_ARG, "need edge > 0, t_run >= 0, min_width > 0");
    const double a = L[0], b = L[1], c = L[3];
    for (int k = 0; k < 9; ++k) h_out[k] = 0.0;
    h_out[8] = edge;
    const M2 cube{edge, 0.0, 0.0, edge};
    if (min_width_over(a, b, c, cube, t_run, 61, 8) >= min_width) {
        h_out[0] = edge;
        h_out[4] = edge;
        if (kind) *kind = LHMM_CELL_CUBIC;
        return LHMM_OK;
    }
    const double k2 = a * a + b * c;
    M2 best{};
    if (k2 <= 0.0) {
        // rotated squares, 46 angles of [0, pi/2)
        double bw = -1.0;
        for (int i = 0; i < 46; ++i) {
            const double th = 0.5 * M_PI * i / 46.0;
            const M2 R{std::cos(th) * edge, -std::sin(th) * edge, std::sin(th) * edge, std::cos(th) * edge};
            const double w = min_width_over(a, b, c, R, t_run, 81, 24);
            if (w > bw) {
                bw = w;
                best = R;
            }
        }
        if (kind) *kind = LHMM_CELL_ROTATED;
    } else {
        const double k = std::sqrt(k2);
        M2 V{};
        eigvec(a, b, c, k, &V.a, &V.c);
        eigvec(a, b, c, -k, &V.b, &V.d);
        const double mu = 0.5 * (3.0 + std::sqrt(5.0));
        const M2 W{1.0, 1.0, mu - 2.0, 1.0 / mu - 2.0};  // eigenvectors of M for mu, 1/mu
        const double dw = det(W);
        const M2 Wi{W.d / dw, -W.b / dw, -W.c / dw, W.a / dw};
        const double T = std::log(mu) / k;
        // The flow maps member r to member r e^{2 k t} (up to scale), so the
        // members are time shifts of one lattice and share its narrowest
        // width over a period, up to the sampling of the period: among the
        // members within 1e-9 of the best, the one widest at t = 0 is taken
        // (the box starts in its widest phase).
        std::vector<std::pair<double, M2>> cands;
        double bw = -1.0;
        for (int sgn = 0; sgn < 2; ++sgn)
            for (int i = 0; i <= 80; ++i) {
                const double r = std::exp(-4.0 + 0.1 * i);
                const M2 D{r, 0.0, 0.0, sgn == 0 ? 1.0 : -1.0};
                M2 P = mul(mul(V, D), Wi);
                const double dp = det(P);
                if (!(std::fabs(dp) > 1e-300)) continue;
                const double s = std::sqrt(edge * edge / std::fabs(dp));
                P = {P.a * s, P.b * s, P.c * s, P.d * s};
                if (det(P) < 0) P = {P.b, P.a, P.d, P.c};
                const double w = min_width_over(a, b, c, P, T, 25, 8);
                cands.push_back({w, P});
                bw = std::max(bw, w);
            }
        double w0 = -1.0;
        for (const auto& cw : cands) {
            if (!(cw.first >= bw * (1.0 - 1e-9))) continue;
            const double w = lattice_min_width(cw.second, 8);
            if (w > w0) {
                w0 = w;
                best = cw.second;
            }
        }
        // the flow over one period maps the lattice onto itself
        const double db = det(best);
        const M2 Pi{best.d / db, -best.b / db, -best.c / db, best.a / db};
        const M2 Mt = mul(mul(Pi, expm(a, b, c, T)), best);
        for (double v : {Mt.a, Mt.b, Mt.c, Mt.d})
            if (std::fabs(v - std::round(v)) > 1e-6) return lhmm_fail(LHMM_ERR_ARG, "no self-mapping lattice found");
        if (kind) *kind = LHMM_CELL_KR;
    }
    M2 red{};
    if (!short_basis(best, &red)) return lhmm_fail(LHMM_ERR_ARG, "degenerate lattice");
    h_out[0] = red.a;
    h_out[1] = red.b;
    h_out[3] = red.c;
    h_out[4] = red.d;
    return LHMM_OK;
}
