/*
 * sph_oracle.c -- double-precision CPU oracle of the SPH macro side of the
 * Lagrangian Heterogeneous Multiscale Method (2-D, periodic box).
 *
 * TEST INFRASTRUCTURE ONLY (see lhmm_oracle.c).  Plain C, all-pairs loops,
 * each quantity computed as the paper writes it:
 *   - number density d_I = sum_J W(r_IJ) (self included) and rho_I = m d_I
 *     (Sec. "Macroscale: Smoothed Particle Hydrodynamics");
 *   - Tait equation of state, Eq. (tait), background pressure
 *     p_b = theta c^2 rho0 / 7;
 *   - momentum equation, Eq. (sph_continuity): pressure, viscous (friction
 *     coefficients a = 2 eta - zeta, b = 4 zeta + 2 eta) and the
 *     micro-to-macro polymer term with <pi>_IJ = pi_I/d_I^2 + pi_J/d_J^2,
 *     plus a body force per unit mass;
 *   - velocity gradient for the micro-domains, Eq. (macro_micro), read with
 *     the volume factor 1/d_J: (grad v)_I = sum_J F_IJ r_IJ (x) v_IJ / d_J;
 *   - velocity-Verlet time stepping (Appendix "Detailed Coupling Protocol",
 *     Step 1);
 *   - solid obstacles (the cylinders of the flow past a periodic array,
 *     Sec. "Flow Past a Periodic Array of Cylinders"), on which the paper
 *     gives no treatment: here the last n_fixed particles are frozen wall
 *     particles that take part in every sum as neighbours (density,
 *     pressure, viscous term with their zero velocity) but never move,
 *     carry no micro-domain and no polymer stress, and get no gradient.
 * Kernels (S_KERNEL), both of support radius h, F_IJ = -W'(r_IJ)/r_IJ:
 *   0: the quintic spline, q = 3 r / h,
 *      W = 63/(478 pi h^2) [(3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5] (terms where
 *      the bracket is positive);
 *   1: the 2-D Lucy kernel of Appendix "Kernel function approximation",
 *      Eq. (lucy_kernel), q = r / h: W = 5/(pi h^2) (1 + 3q) (1 - q)^3 for
 *      q < 1; its derivative is taken by the product rule of that form.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* parameter vector layout (double[S_COUNT]); S_KERNEL: 0 quintic, 1 Lucy;
 * S_MICRO_DIM: 3 for 3-D micro-domains, 2 for planar ones;
 * S_NFIXED: number of trailing
 * wall particles; S_FMODE: 0 = body force +F for y >= Ly/2, -F below
 * (reverse Poiseuille), 1 = +F everywhere */
enum {
    S_RHO0 = 0, S_ETA, S_ZETA, S_C, S_THETA, S_F, S_H, S_DT, S_MASS, S_LX, S_LY, S_LAMBDA, S_ALPHA, S_NFIXED,
    S_FMODE, S_KERNEL, S_MICRO_DIM, S_COUNT
};

static int n_mobile(const double *P, int n) { return n - (int)P[S_NFIXED]; }

static double quintic_W(double r, double h)
{
    double q = 3.0 * r / h;
    if (q >= 3.0) return 0.0;
    double w = pow(3.0 - q, 5);
    if (q < 2.0) w -= 6.0 * pow(2.0 - q, 5);
    if (q < 1.0) w += 15.0 * pow(1.0 - q, 5);
    return 63.0 / (478.0 * M_PI * h * h) * w;
}

/* F = -W'(r)/r, r > 0 */
static double quintic_F(double r, double h)
{
    double q = 3.0 * r / h;
    if (q >= 3.0) return 0.0;
    double dw = -5.0 * pow(3.0 - q, 4);
    if (q < 2.0) dw += 30.0 * pow(2.0 - q, 4);
    if (q < 1.0) dw -= 75.0 * pow(1.0 - q, 4);
    double dWdr = 63.0 / (478.0 * M_PI * h * h) * dw * 3.0 / h;
    return -dWdr / r;
}

static double lucy_W(double r, double h)
{
    double q = r / h;
    if (q >= 1.0) return 0.0;
    return 5.0 / (M_PI * h * h) * (1.0 + 3.0 * q) * pow(1.0 - q, 3);
}

/* d/dr of (1 + 3q)(1 - q)^3 = (3/h)(1 - q)^3 - (3/h)(1 + 3q)(1 - q)^2 */
static double lucy_F(double r, double h)
{
    double q = r / h;
    if (q >= 1.0) return 0.0;
    double dWdr = 5.0 / (M_PI * h * h) * (3.0 / h * pow(1.0 - q, 3) - 3.0 / h * (1.0 + 3.0 * q) * pow(1.0 - q, 2));
    return -dWdr / r;
}

double oracle_sph_W(double r, double h, int kernel) { return kernel == 1 ? lucy_W(r, h) : quintic_W(r, h); }

/* F = -W'(r)/r, r > 0 */
double oracle_sph_F(double r, double h, int kernel) { return kernel == 1 ? lucy_F(r, h) : quintic_F(r, h); }

static double kern_W(const double *P, double r) { return oracle_sph_W(r, P[S_H], (int)P[S_KERNEL]); }
static double kern_F(const double *P, double r) { return oracle_sph_F(r, P[S_H], (int)P[S_KERNEL]); }

static void min_image(const double *P, double *dx, double *dy)
{
    *dx -= P[S_LX] * round(*dx / P[S_LX]);
    *dy -= P[S_LY] * round(*dy / P[S_LY]);
}

/* d (n) and p (n) */
void oracle_sph_density(const double *P, int n, const double *r, double *d, double *p)
{
    const double rho0 = P[S_RHO0], c = P[S_C], m = P[S_MASS];
    const double B = c * c * rho0 / 7.0;
    for (int I = 0; I < n; ++I) {
        double s = 0.0;
        for (int J = 0; J < n; ++J) {
            double dx = r[2 * I] - r[2 * J], dy = r[2 * I + 1] - r[2 * J + 1];
            min_image(P, &dx, &dy);
            s += kern_W(P, sqrt(dx * dx + dy * dy));
        }
        d[I] = s;
        double rho = m * s;
        p[I] = B * (pow(rho / rho0, 7) - 1.0) + P[S_THETA] * B;
    }
}

/* G (n x 4): G_ab = (grad v)_ab = d_a v_b = sum_J F r_a v_b / d_J, row-major */
void oracle_sph_gradv(const double *P, int n, const double *r, const double *v, const double *d, double *G)
{
    const double h = P[S_H];
    for (int I = 0; I < n; ++I) {
        double g[4] = {0, 0, 0, 0};
        for (int J = 0; J < n; ++J) {
            if (J == I) continue;
            double dx = r[2 * I] - r[2 * J], dy = r[2 * I + 1] - r[2 * J + 1];
            min_image(P, &dx, &dy);
            double rr = sqrt(dx * dx + dy * dy);
            if (rr >= h || rr == 0.0) continue;
            double F = kern_F(P, rr) / d[J];
            double vx = v[2 * I] - v[2 * J], vy = v[2 * I + 1] - v[2 * J + 1];
            g[0] += F * dx * vx;
            g[1] += F * dx * vy;
            g[2] += F * dy * vx;
            g[3] += F * dy * vy;
        }
        memcpy(&G[4 * I], g, sizeof g);
    }
}

/* acceleration (n x 2) from Eq. (sph_continuity); pi (n x 3: xx, xy, yy) is
 * the polymer stress already multiplied by alpha / lambda* (rows of wall
 * particles are ignored: walls carry none); body force per S_FMODE.  Wall
 * particles get zero acceleration. */
void oracle_sph_accel(const double *P, int n, const double *r, const double *v, const double *d,
                      const double *p, const double *pi, double *acc)
{
    const double h = P[S_H], m = P[S_MASS];
    const double av = 2.0 * P[S_ETA] - P[S_ZETA], bv = 4.0 * P[S_ZETA] + 2.0 * P[S_ETA];
    const int nm = n_mobile(P, n);
    for (int I = 0; I < n; ++I) {
        if (I >= nm) {
            acc[2 * I] = acc[2 * I + 1] = 0.0;
            continue;
        }
        double fx = 0.0, fy = 0.0;
        for (int J = 0; J < n; ++J) {
            if (J == I) continue;
            double dx = r[2 * I] - r[2 * J], dy = r[2 * I + 1] - r[2 * J + 1];
            min_image(P, &dx, &dy);
            double rr = sqrt(dx * dx + dy * dy);
            if (rr >= h || rr == 0.0) continue;
            double F = kern_F(P, rr);
            double ex = dx / rr, ey = dy / rr;
            double vx = v[2 * I] - v[2 * J], vy = v[2 * I + 1] - v[2 * J + 1];
            /* pressure */
            double pp = p[I] / (d[I] * d[I]) + p[J] / (d[J] * d[J]);
            fx += pp * F * dx;
            fy += pp * F * dy;
            /* viscous */
            double ve = vx * ex + vy * ey;
            double vis = F / (d[I] * d[J]);
            fx -= (av * vx + bv * ve * ex) * vis;
            fy -= (av * vy + bv * ve * ey) * vis;
            /* polymer stress <pi>_IJ . r_IJ F_IJ */
            double i2 = 1.0 / (d[I] * d[I]), j2 = J < nm ? 1.0 / (d[J] * d[J]) : 0.0;
            int Jp = J < nm ? J : I; /* a wall contributes no polymer stress */
            double sxx = pi[3 * I] * i2 + pi[3 * Jp] * j2;
            double sxy = pi[3 * I + 1] * i2 + pi[3 * Jp + 1] * j2;
            double syy = pi[3 * I + 2] * i2 + pi[3 * Jp + 2] * j2;
            fx -= (sxx * dx + sxy * dy) * F;
            fy -= (sxy * dx + syy * dy) * F;
        }
        double body = (P[S_FMODE] != 0.0 || r[2 * I + 1] >= 0.5 * P[S_LY]) ? P[S_F] : -P[S_F];
        acc[2 * I] = fx / m + body;
        acc[2 * I + 1] = fy / m;
    }
}

static double wrapL(double x, double L)
{
    x -= L * floor(x / L);
    if (x >= L) x = 0.0;
    return x;
}

/* One velocity-Verlet step with the polymer stress held fixed; then the
 * velocity gradient at the new state and the micro-domain gradient
 * L_I = lambda* x traceless part of (grad v)^T, as a 3x3 row-major matrix
 * (zero z row and column).  Work arrays: d, p (n), acc (2n). */
void oracle_sph_step(const double *P, int n, double *r, double *v, const double *pi, double *d, double *p,
                     double *acc, double *G, double *Lout)
{
    const double dt = P[S_DT];
    const int nm = n_mobile(P, n);
    oracle_sph_density(P, n, r, d, p);
    oracle_sph_accel(P, n, r, v, d, p, pi, acc);
    for (int k = 0; k < 2 * nm; ++k) v[k] += 0.5 * dt * acc[k];
    for (int I = 0; I < nm; ++I) {
        r[2 * I] = wrapL(r[2 * I] + dt * v[2 * I], P[S_LX]);
        r[2 * I + 1] = wrapL(r[2 * I + 1] + dt * v[2 * I + 1], P[S_LY]);
    }
    oracle_sph_density(P, n, r, d, p);
    oracle_sph_accel(P, n, r, v, d, p, pi, acc);
    for (int k = 0; k < 2 * nm; ++k) v[k] += 0.5 * dt * acc[k];
    oracle_sph_gradv(P, n, r, v, d, G);
    for (int I = 0; I < n; ++I) {
        if (I >= nm) {
            for (int k = 0; k < 9; ++k) Lout[9 * I + k] = 0.0;
            continue;
        }
        const double *g = &G[4 * I];
        /* u = L r with L = (grad v)^T: L = [[g0, g2], [g1, g3]] */
        double L00 = g[0], L01 = g[2], L10 = g[1], L11 = g[3];
        double half_tr = 0.5 * (L00 + L11);
        double *o = &Lout[9 * I];
        for (int k = 0; k < 9; ++k) o[k] = 0.0;
        o[0] = P[S_LAMBDA] * (L00 - half_tr);
        o[1] = P[S_LAMBDA] * L01;
        o[3] = P[S_LAMBDA] * L10;
        o[4] = P[S_LAMBDA] * (L11 - half_tr);
    }
}

/* polymer stress for the macro side from the micro-domains' mean stress
 * (n x 6: xx, yy, zz, xy, xz, yz), Eq. (pip): alpha / lambda* x the in-plane
 * components of the deviatoric stress, as (xx, xy, yy).  The deviatoric
 * part of a 3-D micro stress removes its isotropic part tr/3; a planar
 * micro-domain (S_MICRO_DIM = 2) has no zz stress, and its deviatoric part
 * is taken in its own plane, removing (xx + yy)/2. */
void oracle_sph_polymer_stress(const double *P, int n, const double *sig, double *pi)
{
    const double s = P[S_ALPHA] / P[S_LAMBDA];
    const int planar = (int)P[S_MICRO_DIM] == 2;
    for (int I = 0; I < n; ++I) {
        const double *g = &sig[6 * I];
        double iso = planar ? (g[0] + g[1]) / 2.0 : (g[0] + g[1] + g[2]) / 3.0;
        pi[3 * I] = s * (g[0] - iso);
        pi[3 * I + 1] = s * g[3];
        pi[3 * I + 2] = s * (g[1] - iso);
    }
}
