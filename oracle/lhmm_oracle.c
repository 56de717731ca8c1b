/*
 * lhmm_oracle.c -- double-precision CPU oracle for the micro-DPD hot path of
 * the Lagrangian Heterogeneous Multiscale Method (one periodic DPD/FENE
 * micro-box per SPH macro particle, driven by that particle's velocity
 * gradient, returning the Irving-Kirkwood stress).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP path; it is plain C in double
 * precision, with every step taken in the order the method states it.
 *
 * What each part follows (paper sections / equations):
 *   - pair forces: Sec. "Microscale: Polymer Melt Model -- DPD and FENE",
 *     Eqs. (F_DPD), (conservative), (dissipative), (random), with the
 *     fluctuation-dissipation relation stated after Eq. (random);
 *   - bond force: Eq. (fene_force), read as attractive (minus the gradient
 *     of U = -1/2 H R0^2 ln(1 - r^2/R0^2));
 *   - equation of motion: Eq. (motion), integrated by velocity-Verlet
 *     (Appendix "Detailed Coupling Protocol", Step 3);
 *   - stress: Eqs. (IKtotal), (kinetic_stress), (potential_stress).  With a
 *     uniform weight over the whole periodic cell the bond function equals
 *     1/V and the Irving-Kirkwood stress is the cell's virial stress;
 *   - imposed flow: Sec. "Macro-to-Micro Coupling", Eq. (micro_bc) imposes
 *     v = L r.  Two forms: homogeneously, the periodic cell deforming with
 *     dh/dt = L h and particles carrying peculiar velocities c = v - L r
 *     (oracle_run_box); or, as the paper's micro-domain does (Tab. 2), on
 *     the boundary-condition ring of a fixed cell only, with the stress
 *     sampled over the core (oracle_run_box_afbc).
 *
 * Readings taken where the paper is silent or garbled:
 *   - the discrete random force carries 1/sqrt(dt);
 *   - w^R(r) = 1 - r/rc and w^D = (w^R)^2; sigma = sqrt(2 gamma kBT);
 *   - bonded pairs also feel the DPD pair forces (the sum in Eq. F_DPD runs
 *     over all j != i);
 *   - stress is tension-positive: sigma = -(sum m c c + sum_pairs d f)/V;
 *   - theta_ij is a Box-Muller normal from Philox4x32-10 (Salmon et al.,
 *     SC'11) with counter (min id, max id, step, box), key (seed lo, seed hi);
 *   - a bond reaching r >= R0 raises a sticky BOND flag and its denominator
 *     is clamped at 0.01;
 *   - the in-plane cell basis is kept Lagrange-Gauss reduced; a perpendicular
 *     width below 3 rc raises a sticky CELL flag;
 *   - boundary regions: a particle's position r' is taken relative to the
 *     cell's centre (the domain's mean velocity is removed, so its centre of
 *     mass stays there); the regions are squares in the plane; on the
 *     boundary-condition ring the in-plane velocity relaxes, after each half
 *     kick, toward the imposed field of Eq. (micro_bc) at rate zeta with the
 *     matching thermal noise (an Ornstein-Uhlenbeck step), so the ring's mean
 *     flow is v' = G r' while its particles keep kBT and feel the forces (a
 *     velocity overwritten with G r' would freeze the ring's particles in
 *     place and let it absorb the core's); the noise is a Box-Muller pair
 *     from Philox4x32-10 with counter (id, 0xFFFFFFF0 + half kick, step,
 *     box); the weight of the Irving-Kirkwood stress is uniform over the
 *     core and zero outside, so the kinetic part sums the core's particles
 *     (velocity relative to the imposed field) and a pair's bond function
 *     is the fraction of its segment inside the core over the core's volume.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_ERR_BOND 1u
#define ORACLE_ERR_CELL 2u
#define ORACLE_ERR_NONFINITE 4u
#define ORACLE_ERR_ARG 8u

/* parameter vector layout (double[9]) */
enum { P_A = 0, P_GAMMA, P_SIGMA, P_KBT, P_MASS, P_RC, P_DT, P_H, P_R0, P_COUNT };

/* stress component order: xx, yy, zz, xy, xz, yz */
static const int SI[6] = {0, 1, 2, 0, 0, 1};
static const int SJ[6] = {0, 1, 2, 1, 2, 2};

/* --------------------------------------------------------------------- */
/* Counter-based random numbers                                          */
/* --------------------------------------------------------------------- */

/* Philox4x32 with 10 rounds, as published by Salmon, Moraes, Dror and Shaw
 * ("Parallel random numbers: as easy as 1, 2, 3", SC'11): each round
 * multiplies words 0 and 2 by two fixed odd constants, keeps the 64-bit
 * products' halves, permutes and xors with the round key; the key is bumped
 * by the Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1) from the top 23 bits of a word: (2 m + 1) / 2^24.
 * Every value is exact in single and in double precision. */
double oracle_uniform23(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* theta_ij of Eq. (random): a unit normal that is symmetric in (i, j) and
 * fresh at every step, by Box-Muller on two uniforms of one Philox block. */
double oracle_theta(uint64_t seed, uint32_t id_i, uint32_t id_j, uint32_t step, uint32_t box)
{
    uint32_t ctr[4], key[2], x[4];
    ctr[0] = id_i < id_j ? id_i : id_j;
    ctr[1] = id_i < id_j ? id_j : id_i;
    ctr[2] = step;
    ctr[3] = box;
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, x);
    double u0 = oracle_uniform23(x[0]);
    double u1 = oracle_uniform23(x[1]);
    return sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
}

/* --------------------------------------------------------------------- */
/* Cell algebra (row-major 3x3; columns of h are the lattice vectors)    */
/* --------------------------------------------------------------------- */

static void mat_mul(const double A[9], const double B[9], double C[9])
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = acc;
        }
    memcpy(C, T, sizeof(T));
}

static void mat_vec(const double A[9], const double x[3], double y[3])
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}

static double mat_det(const double A[9])
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void mat_inv(const double A[9], double B[9])
{
    double det = mat_det(A);
    double T[9];
    T[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    T[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    T[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    T[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    T[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    T[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    T[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    T[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    T[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    memcpy(B, T, sizeof(T));
}

/* Is L an in-plane (x-y), traceless velocity gradient?  Returns 1 if so. */
int oracle_check_gradient(const double L[9])
{
    double scale = 1.0;
    for (int k = 0; k < 9; ++k) {
        if (!isfinite(L[k])) return 0;
        scale += fabs(L[k]);
    }
    if (L[2] != 0.0 || L[5] != 0.0 || L[6] != 0.0 || L[7] != 0.0 || L[8] != 0.0) return 0;
    if (fabs(L[0] + L[4]) > 1e-12 * scale) return 0;
    return 1;
}

/* E = exp(L tau) for an in-plane traceless L.  In the plane L^2 = k^2 I with
 * k^2 = a^2 + b c (Cayley-Hamilton), so exp(L tau) = f0 I + f1 L with
 * (cosh, sinh/k), (cos, sin/w) or (1, tau) for k^2 >, <, = 0.  The z row
 * and column of E are those of the identity. */
void oracle_expL(const double L[9], double tau, double E[9])
{
    double a = 0.5 * (L[0] - L[4]);
    double b = L[1], c = L[3];
    double k2 = a * a + b * c;
    double f0, f1;
    if (k2 > 0.0) {
        double k = sqrt(k2);
        f0 = cosh(k * tau);
        f1 = sinh(k * tau) / k;
    } else if (k2 < 0.0) {
        double w = sqrt(-k2);
        f0 = cos(w * tau);
        f1 = sin(w * tau) / w;
    } else {
        f0 = 1.0;
        f1 = tau;
    }
    E[0] = f0 + f1 * a; E[1] = f1 * b;      E[2] = 0.0;
    E[3] = f1 * c;      E[4] = f0 - f1 * a; E[5] = 0.0;
    E[6] = 0.0;         E[7] = 0.0;         E[8] = 1.0;
}

/* Perpendicular widths of the cell: w_a = V / |h_b x h_c|. */
void oracle_widths(const double h[9], double w[3])
{
    double col[3][3];
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) col[a][r] = h[3 * r + a];
    double V = fabs(mat_det(h));
    for (int a = 0; a < 3; ++a) {
        const double *u = col[(a + 1) % 3], *v = col[(a + 2) % 3];
        double x = u[1] * v[2] - u[2] * v[1];
        double y = u[2] * v[0] - u[0] * v[2];
        double z = u[0] * v[1] - u[1] * v[0];
        w[a] = V / sqrt(x * x + y * y + z * z);
    }
}

/* Lagrange-Gauss reduction of the in-plane basis (b1, b2) = first two
 * columns of h.  Swaps are taken as (b1, b2) -> (b2, -b1) and size
 * reductions as b2 -> b2 - m b1 with m = floor(mu + 1/2), so the integer
 * matrix U (h_new = h U, det U = +1) is accumulated.  Returns 1 if the
 * basis changed.  U is row-major 2x2. */
int oracle_reduce_cell(double h[9], int U[4])
{
    double b1[2] = {h[0], h[3]}, b2[2] = {h[1], h[4]};
    long u00 = 1, u01 = 0, u10 = 0, u11 = 1;
    int changed = 0;
    for (int iter = 0; iter < 256; ++iter) {
        double n1 = b1[0] * b1[0] + b1[1] * b1[1];
        double n2 = b2[0] * b2[0] + b2[1] * b2[1];
        if (n2 < n1) {
            double t0 = b1[0], t1 = b1[1];
            b1[0] = b2[0]; b1[1] = b2[1];
            b2[0] = -t0;   b2[1] = -t1;
            /* U <- U [[0,-1],[1,0]] */
            long a0 = u01, a1 = -u00, c0 = u11, c1 = -u10;
            u00 = a0; u01 = a1; u10 = c0; u11 = c1;
            changed = 1;
            continue;
        }
        double mu = (b1[0] * b2[0] + b1[1] * b2[1]) / n1;
        long m = (long)floor(mu + 0.5);
        if (m == 0) break;
        b2[0] -= (double)m * b1[0];
        b2[1] -= (double)m * b1[1];
        /* U <- U [[1,-m],[0,1]] */
        u01 -= m * u00;
        u11 -= m * u10;
        changed = 1;
    }
    h[0] = b1[0]; h[3] = b1[1];
    h[1] = b2[0]; h[4] = b2[1];
    U[0] = (int)u00; U[1] = (int)u01; U[2] = (int)u10; U[3] = (int)u11;
    return changed;
}

/* --------------------------------------------------------------------- */
/* Pair search                                                            */
/* --------------------------------------------------------------------- */

typedef struct {
    int i, j;
    double d[3]; /* r_i - r_j, the image within the cutoff */
} opair;

typedef struct {
    opair *p;
    long n, cap;
} opairs;

static void pairs_push(opairs *P, int i, int j, const double d[3])
{
    if (P->n == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 1024;
        P->p = (opair *)realloc(P->p, (size_t)P->cap * sizeof(opair));
    }
    P->p[P->n].i = i;
    P->p[P->n].j = j;
    P->p[P->n].d[0] = d[0];
    P->p[P->n].d[1] = d[1];
    P->p[P->n].d[2] = d[2];
    P->n++;
}

/* The definition: every unordered pair i < j and every periodic image of j
 * around the nearest fractional one; pairs with 0 < r < rc are kept. */
static void pairs_brute(int N, const double *s, const double h[9], double rc, opairs *out)
{
    double rc2 = rc * rc;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) {
            double ds0[3];
            for (int a = 0; a < 3; ++a) {
                ds0[a] = s[3 * i + a] - s[3 * j + a];
                ds0[a] -= floor(ds0[a] + 0.5);
            }
            for (int n0 = -1; n0 <= 1; ++n0)
                for (int n1 = -1; n1 <= 1; ++n1)
                    for (int n2 = -1; n2 <= 1; ++n2) {
                        double ds[3] = {ds0[0] + n0, ds0[1] + n1, ds0[2] + n2}, d[3];
                        mat_vec(h, ds, d);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rc2 && r2 > 0.0) pairs_push(out, i, j, d);
                    }
        }
}

/* The same set found through a grid of n_a = floor(w_a / rc) cells along
 * each fractional axis (valid when every n_a >= 3): a particle within rc of
 * i lies in one of the 27 cells around i's cell. */
static int pairs_cells(int N, const double *s, const double h[9], double rc, opairs *out)
{
    double w[3];
    int n[3];
    oracle_widths(h, w);
    for (int a = 0; a < 3; ++a) {
        n[a] = (int)floor(w[a] / rc);
        if (n[a] < 3) return -1;
    }
    long ncell = (long)n[0] * n[1] * n[2];
    int *head = (int *)malloc((size_t)ncell * sizeof(int));
    int *next = (int *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int));
    int *cell = (int *)malloc((size_t)(N > 0 ? 3 * N : 3) * sizeof(int));
    for (long k = 0; k < ncell; ++k) head[k] = -1;
    /* insert in descending order so each cell's list is ascending in id */
    for (int i = N - 1; i >= 0; --i) {
        for (int a = 0; a < 3; ++a) {
            int k = (int)floor(s[3 * i + a] * n[a]);
            if (k < 0) k = 0;
            if (k >= n[a]) k = n[a] - 1;
            cell[3 * i + a] = k;
        }
        long id = ((long)cell[3 * i] * n[1] + cell[3 * i + 1]) * n[2] + cell[3 * i + 2];
        next[i] = head[id];
        head[id] = i;
    }
    double rc2 = rc * rc;
    for (int i = 0; i < N; ++i) {
        for (int d0 = -1; d0 <= 1; ++d0)
            for (int d1 = -1; d1 <= 1; ++d1)
                for (int d2 = -1; d2 <= 1; ++d2) {
                    int dd[3] = {d0, d1, d2}, m[3];
                    double shift[3];
                    for (int a = 0; a < 3; ++a) {
                        m[a] = cell[3 * i + a] + dd[a];
                        shift[a] = 0.0;
                        if (m[a] < 0) { m[a] += n[a]; shift[a] = -1.0; }
                        if (m[a] >= n[a]) { m[a] -= n[a]; shift[a] = 1.0; }
                    }
                    long id = ((long)m[0] * n[1] + m[1]) * n[2] + m[2];
                    for (int j = head[id]; j >= 0; j = next[j]) {
                        if (j <= i) continue;
                        double ds[3], d[3];
                        for (int a = 0; a < 3; ++a) ds[a] = s[3 * i + a] - (s[3 * j + a] + shift[a]);
                        mat_vec(h, ds, d);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rc2 && r2 > 0.0) pairs_push(out, i, j, d);
                    }
                }
    }
    free(head);
    free(next);
    free(cell);
    return 0;
}

/* Pair list for tests: mode 0 = brute force, 1 = cell grid.  Writes up to
 * max_pairs (i, j) and the displacement; returns the count (or -1 if the
 * cell grid is not applicable). */
long oracle_pairs(int N, const double *s, const double h[9], double rc, int mode, int *ij, double *d,
                  long max_pairs)
{
    opairs P = {0, 0, 0};
    if (mode == 0)
        pairs_brute(N, s, h, rc, &P);
    else if (pairs_cells(N, s, h, rc, &P) != 0) {
        free(P.p);
        return -1;
    }
    for (long k = 0; k < P.n && k < max_pairs; ++k) {
        ij[2 * k] = P.p[k].i;
        ij[2 * k + 1] = P.p[k].j;
        for (int a = 0; a < 3; ++a) d[3 * k + a] = P.p[k].d[a];
    }
    long n = P.n;
    free(P.p);
    return n;
}

/* --------------------------------------------------------------------- */
/* Forces and virial                                                      */
/* --------------------------------------------------------------------- */

double oracle_core_fraction(const double a[2], const double b[2], double hc);

/* in-plane position of fractional coordinate s relative to the cell centre */
static void centred(const double h[9], const double *s, double out[2])
{
    out[0] = h[0] * (s[0] - 0.5) + h[1] * (s[1] - 0.5);
    out[1] = h[3] * (s[0] - 0.5) + h[4] * (s[1] - 0.5);
}

/* F (N x 3) and the virial sum_pairs d (x) f of each part:
 * W[0] conservative, W[1] dissipative, W[2] random, W[3] FENE (6 comps each).
 * Particles 0 .. n_chains*chain_len-1 form chains of chain_len consecutive
 * ids; the rest are solvent.  mode: 0 brute force, 1 cell grid (falls back
 * to brute force when the grid has fewer than 3 cells along an axis).
 * hc >= 0: each pair's (and bond's) virial term is weighted by the
 * fraction of its segment inside the core |x'|, |y'| <= hc (positions
 * relative to the cell centre), the bond function of Eq. (potential_stress)
 * for a weight uniform over the core, times the core's volume. */
static int forces_impl(const double *P, uint64_t seed, int chain_len, uint32_t box, int N, int n_chains,
                       const double *s, const double *c, const double h[9], const double L[9], uint32_t step,
                       double *F, double W[24], uint32_t *err, int mode, long long *npairs, double hc)
{
    const double a = P[P_A], gamma = P[P_GAMMA], sigma = P[P_SIGMA], rc = P[P_RC], dt = P[P_DT];
    const double Hf = P[P_H], R0 = P[P_R0];
    const double rdt = 1.0 / sqrt(dt);
    for (int k = 0; k < 3 * N; ++k) F[k] = 0.0;
    for (int k = 0; k < 24; ++k) W[k] = 0.0;

    opairs pl = {0, 0, 0};
    if (mode == 0 || pairs_cells(N, s, h, rc, &pl) != 0) {
        pl.n = 0;
        pairs_brute(N, s, h, rc, &pl);
    }
    if (npairs) *npairs += pl.n;
    for (long q = 0; q < pl.n; ++q) {
        int i = pl.p[q].i, j = pl.p[q].j;
        const double *d = pl.p[q].d;
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double e[3] = {d[0] / r, d[1] / r, d[2] / r};
        double wR = 1.0 - r / rc;
        double wD = wR * wR;
        /* relative velocity of i and the image of j: peculiar parts plus the
         * streaming difference L d */
        double Ld[3];
        mat_vec(L, d, Ld);
        double v[3];
        for (int k = 0; k < 3; ++k) v[k] = c[3 * i + k] - c[3 * j + k] + Ld[k];
        double ev = e[0] * v[0] + e[1] * v[1] + e[2] * v[2];
        double th = oracle_theta(seed, (uint32_t)i, (uint32_t)j, step, box);
        double mag[3];
        mag[0] = a * wR;                  /* conservative */
        mag[1] = -gamma * wD * ev;        /* dissipative  */
        mag[2] = sigma * wR * th * rdt;   /* random       */
        double wgt = 1.0;
        if (hc >= 0.0) {
            double ri[2], rj[2];
            centred(h, &s[3 * i], ri);
            rj[0] = ri[0] - d[0];
            rj[1] = ri[1] - d[1];
            wgt = oracle_core_fraction(ri, rj, hc);
        }
        for (int part = 0; part < 3; ++part) {
            double f[3] = {mag[part] * e[0], mag[part] * e[1], mag[part] * e[2]};
            for (int k = 0; k < 3; ++k) {
                F[3 * i + k] += f[k];
                F[3 * j + k] -= f[k];
            }
            for (int q6 = 0; q6 < 6; ++q6) W[6 * part + q6] += wgt * d[SI[q6]] * f[SJ[q6]];
        }
    }
    free(pl.p);

    /* FENE springs between consecutive beads of each chain */
    for (int ch = 0; ch < n_chains; ++ch)
        for (int b = 0; b + 1 < chain_len; ++b) {
            int i = ch * chain_len + b, j = i + 1;
            double ds0[3], best[3] = {0, 0, 0}, bestr2 = INFINITY;
            for (int k = 0; k < 3; ++k) {
                ds0[k] = s[3 * i + k] - s[3 * j + k];
                ds0[k] -= floor(ds0[k] + 0.5);
            }
            for (int n0 = -1; n0 <= 1; ++n0)
                for (int n1 = -1; n1 <= 1; ++n1)
                    for (int n2 = -1; n2 <= 1; ++n2) {
                        double ds[3] = {ds0[0] + n0, ds0[1] + n1, ds0[2] + n2}, d[3];
                        mat_vec(h, ds, d);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < bestr2) {
                            bestr2 = r2;
                            best[0] = d[0]; best[1] = d[1]; best[2] = d[2];
                        }
                    }
            double den = 1.0 - bestr2 / (R0 * R0);
            if (den <= 0.0) *err |= ORACLE_ERR_BOND;
            if (den < 0.01) den = 0.01;
            double f[3] = {-Hf * best[0] / den, -Hf * best[1] / den, -Hf * best[2] / den};
            for (int k = 0; k < 3; ++k) {
                F[3 * i + k] += f[k];
                F[3 * j + k] -= f[k];
            }
            double wgt = 1.0;
            if (hc >= 0.0) {
                double ri[2], rj[2];
                centred(h, &s[3 * i], ri);
                rj[0] = ri[0] - best[0];
                rj[1] = ri[1] - best[1];
                wgt = oracle_core_fraction(ri, rj, hc);
            }
            for (int q6 = 0; q6 < 6; ++q6) W[18 + q6] += wgt * best[SI[q6]] * f[SJ[q6]];
        }
    return 0;
}

int oracle_forces(const double *P, uint64_t seed, int chain_len, uint32_t box, int N, int n_chains,
                  const double *s, const double *c, const double h[9], const double L[9], uint32_t step,
                  double *F, double W[24], uint32_t *err, int mode, long long *npairs)
{
    return forces_impl(P, seed, chain_len, box, N, n_chains, s, c, h, L, step, F, W, err, mode, npairs, -1.0);
}


/* --------------------------------------------------------------------- */
/* Time stepping                                                          */
/* --------------------------------------------------------------------- */

static void wrap01(double *x)
{
    *x -= floor(*x);
    if (*x >= 1.0) *x = 0.0;
}

/* Advance one box by nsteps velocity-Verlet steps under a constant velocity
 * gradient L (u = L r).  State: s (N x 3 fractional), c (N x 3 peculiar
 * velocity), F (N x 3 forces at the current state, valid if *fvalid),
 * h (cell), *step (completed steps; the force evaluation that ends step n
 * uses random-number step n).  Outputs: mean stress over the steps
 * (xx,yy,zz,xy,xz,yz), its parts (kinetic, conservative, dissipative,
 * random, FENE; 5 x 6), optionally the per-step stress series (nsteps x 6),
 * and sticky error bits. */
int oracle_run_box(const double *P, uint64_t seed, int chain_len, uint32_t box, int N, int n_chains,
                   double *s, double *c, double *F, int *fvalid, double h[9], uint64_t *step,
                   const double L[9], int nsteps, double *stress_mean, double *parts_mean, double *series,
                   uint32_t *err, int mode, long long *npairs)
{
    const double m = P[P_MASS], dt = P[P_DT], rc = P[P_RC];
    double W[24];
    if (!oracle_check_gradient(L) || nsteps <= 0) {
        *err |= ORACLE_ERR_ARG;
        return -1;
    }
    /* every call starts from zero mean peculiar velocity: the micro-domain
     * moves with its macro particle (pair forces cancel, so under a
     * compressing gradient the mean would follow d<c>/dt = -L <c>) */
    if (N > 0) {
        double mean[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) mean[k] += c[3 * i + k];
        for (int k = 0; k < 3; ++k) mean[k] /= N;
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) c[3 * i + k] -= mean[k];
    }
    if (!*fvalid) {
        oracle_forces(P, seed, chain_len, box, N, n_chains, s, c, h, L, (uint32_t)*step, F, W, err, mode, NULL);
        *fvalid = 1;
    }
    double E[9], Eh[9];
    oracle_expL(L, dt, E);
    oracle_expL(L, 0.5 * dt, Eh);
    double acc[30];
    for (int k = 0; k < 30; ++k) acc[k] = 0.0;

    for (int n = 0; n < nsteps; ++n) {
        /* first half kick: c += dt/2 (F/m - L c) */
        for (int i = 0; i < N; ++i) {
            double Lc[3];
            mat_vec(L, &c[3 * i], Lc);
            for (int k = 0; k < 3; ++k) c[3 * i + k] += 0.5 * dt * (F[3 * i + k] / m - Lc[k]);
        }
        /* drift in fractional coordinates with the mid-step cell */
        double hm[9], hmi[9];
        mat_mul(Eh, h, hm);
        mat_inv(hm, hmi);
        for (int i = 0; i < N; ++i) {
            double ds[3];
            mat_vec(hmi, &c[3 * i], ds);
            for (int k = 0; k < 3; ++k) s[3 * i + k] += dt * ds[k];
        }
        /* deform the cell, keep it reduced, remap and wrap */
        mat_mul(E, h, h);
        int U[4];
        if (oracle_reduce_cell(h, U)) {
            /* s <- U^{-1} s in the plane; U^{-1} = [[u11,-u01],[-u10,u00]] */
            for (int i = 0; i < N; ++i) {
                double x = s[3 * i], y = s[3 * i + 1];
                s[3 * i] = U[3] * x - U[1] * y;
                s[3 * i + 1] = -U[2] * x + U[0] * y;
            }
        }
        for (int k = 0; k < 3 * N; ++k) wrap01(&s[k]);
        *step += 1;
        double w[3];
        oracle_widths(h, w);
        if (w[0] < 3.0 * rc || w[1] < 3.0 * rc || w[2] < 3.0 * rc) *err |= ORACLE_ERR_CELL;

        oracle_forces(P, seed, chain_len, box, N, n_chains, s, c, h, L, (uint32_t)*step, F, W, err, mode,
                      npairs);

        /* second half kick */
        for (int i = 0; i < N; ++i) {
            double Lc[3];
            mat_vec(L, &c[3 * i], Lc);
            for (int k = 0; k < 3; ++k) c[3 * i + k] += 0.5 * dt * (F[3 * i + k] / m - Lc[k]);
        }
        /* stress sample: sigma = -(K + W) / V */
        double K[6] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < N; ++i)
            for (int q6 = 0; q6 < 6; ++q6) K[q6] += m * c[3 * i + SI[q6]] * c[3 * i + SJ[q6]];
        double V = fabs(mat_det(h));
        double sig[6];
        for (int q6 = 0; q6 < 6; ++q6) {
            double tot = K[q6] + W[q6] + W[6 + q6] + W[12 + q6] + W[18 + q6];
            sig[q6] = -tot / V;
            acc[q6] += -K[q6] / V;
            for (int part = 0; part < 4; ++part) acc[6 * (part + 1) + q6] += -W[6 * part + q6] / V;
            if (!isfinite(sig[q6])) *err |= ORACLE_ERR_NONFINITE;
        }
        if (series)
            for (int q6 = 0; q6 < 6; ++q6) series[6 * n + q6] = sig[q6];
    }
    for (int q6 = 0; q6 < 6; ++q6) {
        double tot = 0.0;
        for (int part = 0; part < 5; ++part) tot += acc[6 * part + q6];
        if (stress_mean) stress_mean[q6] = tot / nsteps;
    }
    if (parts_mean)
        for (int k = 0; k < 30; ++k) parts_mean[k] = acc[k] / nsteps;
    return 0;
}

/* Many independent boxes, one OpenMP task per box.  Particle arrays are the
 * boxes' arrays concatenated (box b owns rows off[b] .. off[b+1]-1); h, L
 * are n_boxes x 9; outputs are n_boxes x 6 and n_boxes x 30.  box_ids gives
 * the id each box uses in the random-number counter. */
int oracle_run_batch(const double *P, uint64_t seed, int chain_len, int n_boxes, const int *off,
                     const int *n_chains, const uint32_t *box_ids, double *s, double *c, double *F,
                     int *fvalid, double *h, uint64_t *step, const double *L, int nsteps,
                     double *stress_mean, double *parts_mean, uint32_t *err, int mode, long long *npairs)
{
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : status)
    for (int b = 0; b < n_boxes; ++b) {
        int o = off[b], N = off[b + 1] - off[b];
        int rc = oracle_run_box(P, seed, chain_len, box_ids[b], N, n_chains[b], s + 3 * (long)o,
                                c + 3 * (long)o, F + 3 * (long)o, &fvalid[b], h + 9 * b, &step[b],
                                L + 9 * b, nsteps, stress_mean ? stress_mean + 6 * b : NULL,
                                parts_mean ? parts_mean + 30 * b : NULL, NULL, &err[b], mode,
                                npairs ? &npairs[b] : NULL);
        if (rc != 0) status = 1;
    }
    return status ? -1 : 0;
}

/* --------------------------------------------------------------------- */
/* Micro-domain with adaptive boundary regions                           */
/* --------------------------------------------------------------------- */

/* The micro-domain of Sec. "Macro-to-Micro Coupling" and Tab. 2: a periodic
 * cell split, by the in-plane position r' of a particle relative to the
 * cell's centre, into the core |x'|, |y'| < hc, the boundary-condition ring
 * hc <= max(|x'|, |y'|) < hb and the buffer outside it.  The cell itself
 * does not deform; in the boundary-condition ring every particle's
 * velocity is the imposed field of Eq. (micro_bc), v' = G r' (G = lambda*
 * (grad v)^T, u = G r); the core and the buffer move freely.  The stress is
 * the Irving-Kirkwood stress of Eqs. (IKtotal), (kinetic_stress),
 * (potential_stress) with a weight uniform over the core and zero outside:
 * the kinetic part sums the core's particles with their velocity relative to
 * the imposed field, and the bond function of a pair (or bond) is the
 * fraction of the segment joining the two particles that lies inside the
 * core, over the core's volume. */

/* region of an in-plane position relative to the cell centre: 0 core,
 * 1 boundary-condition ring, 2 buffer */
int oracle_afbc_region(double x, double y, double hc, double hb)
{
    double m = fmax(fabs(x), fabs(y));
    return m < hc ? 0 : (m < hb ? 1 : 2);
}

/* Fraction of the segment from a to b (in-plane) inside the square
 * |x|, |y| <= hc: the bond function of a uniform core weight times the
 * core's volume.  Parametrise p(t) = a + t (b - a), t in [0, 1], and keep
 * the t where both coordinates are within the square. */
double oracle_core_fraction(const double a[2], const double b[2], double hc)
{
    double t0 = 0.0, t1 = 1.0;
    for (int k = 0; k < 2; ++k) {
        double dk = b[k] - a[k];
        if (dk == 0.0) {
            if (a[k] < -hc || a[k] > hc) return 0.0;
            continue;
        }
        double ta = (-hc - a[k]) / dk, tb = (hc - a[k]) / dk;
        if (ta > tb) {
            double x = ta;
            ta = tb;
            tb = x;
        }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    return t1 > t0 ? t1 - t0 : 0.0;
}

/* the pair of standard normals (Box-Muller, cosine and sine branches) that
 * particle id draws at half kick `half` of the step ending at `step` */
void oracle_afbc_noise(uint64_t seed, uint32_t id, uint32_t half, uint32_t step, uint32_t box, double xi[2])
{
    uint32_t ctr[4] = {id, 0xFFFFFFF0u + half, step, box}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    double r = sqrt(-2.0 * log(oracle_uniform23(out[0])));
    xi[0] = r * cos(2.0 * M_PI * oracle_uniform23(out[1]));
    xi[1] = r * sin(2.0 * M_PI * oracle_uniform23(out[1]));
}

/* the ring's in-plane velocities relax toward the imposed field over half a
 * step: c <- u + (c - u) exp(-zeta dt/2) + sqrt(kBT/m (1 - exp(-zeta dt))) xi,
 * u = G r' (an exact Ornstein-Uhlenbeck step of dc = -zeta (c - u) dt + noise) */
static void afbc_relax(const double *P, uint64_t seed, uint32_t box, uint32_t step, uint32_t half, int N,
                       const double *s, double *c, const double h[9], const double G[9], double hc, double hb,
                       double zeta)
{
    const double dt = P[P_DT], kT = P[P_KBT], m = P[P_MASS];
    const double damp = exp(-0.5 * zeta * dt), amp = sqrt(kT / m * (1.0 - exp(-zeta * dt)));
    for (int i = 0; i < N; ++i) {
        double x = h[0] * (s[3 * i] - 0.5) + h[1] * (s[3 * i + 1] - 0.5);
        double y = h[3] * (s[3 * i] - 0.5) + h[4] * (s[3 * i + 1] - 0.5);
        if (oracle_afbc_region(x, y, hc, hb) != 1) continue;
        double u[2] = {G[0] * x + G[1] * y, G[3] * x + G[4] * y}, xi[2];
        oracle_afbc_noise(seed, (uint32_t)i, half, step, box, xi);
        for (int k = 0; k < 2; ++k) c[3 * i + k] = u[k] + (c[3 * i + k] - u[k]) * damp + amp * xi[k];
    }
}

/* Advance one micro-domain with boundary regions (core half-width hc,
 * boundary-condition ring out to half-width hb, relaxation rate zeta of the
 * ring toward the imposed field) by nsteps velocity-Verlet steps under the
 * imposed gradient G; the cell h stays fixed and c is the particles'
 * velocity.  Each step: half kick c += dt/2 F/m, the ring's relaxation,
 * drift s += dt h^-1 c and wrap, forces, half kick, the ring's relaxation
 * again, then the core's stress sample
 *   sigma = -(sum_{i in core} m dv_i (x) dv_i + sum_pairs f_frac d (x) f) / V_core,
 * dv_i = c_i - G r'_i, f_frac the fraction of the pair's segment inside the
 * core, V_core = (2 hc)^2 h_zz.  Outputs as oracle_run_box (mean stress,
 * parts kinetic, conservative, dissipative, random, FENE). */
int oracle_run_box_afbc(const double *P, uint64_t seed, int chain_len, uint32_t box, int N, int n_chains,
                        double *s, double *c, double *F, int *fvalid, const double h[9], uint64_t *step,
                        const double G[9], double hc, double hb, double zeta, int nsteps,
                        double *stress_mean, double *parts_mean, uint32_t *err, int mode)
{
    const double m = P[P_MASS], dt = P[P_DT];
    const double L0[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double W[24];
    if (!oracle_check_gradient(G) || nsteps <= 0 || !(hc > 0.0) || !(hb >= hc) || !(zeta >= 0.0)) {
        *err |= ORACLE_ERR_ARG;
        return -1;
    }
    if (N > 0) {
        double mean[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) mean[k] += c[3 * i + k];
        for (int k = 0; k < 3; ++k) mean[k] /= N;
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) c[3 * i + k] -= mean[k];
    }
    if (!*fvalid) {
        forces_impl(P, seed, chain_len, box, N, n_chains, s, c, h, L0, (uint32_t)*step, F, W, err, mode, NULL,
                    -1.0);
        *fvalid = 1;
    }
    double hi[9];
    mat_inv(h, hi);
    const double Vc = 4.0 * hc * hc * h[8];
    double acc[30];
    for (int k = 0; k < 30; ++k) acc[k] = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        const uint32_t st = (uint32_t)(*step + 1);  /* the step being made */
        for (int k = 0; k < 3 * N; ++k) c[k] += 0.5 * dt * F[k] / m;
        afbc_relax(P, seed, box, st, 0, N, s, c, h, G, hc, hb, zeta);
        for (int i = 0; i < N; ++i) {
            double ds[3];
            mat_vec(hi, &c[3 * i], ds);
            for (int k = 0; k < 3; ++k) s[3 * i + k] += dt * ds[k];
        }
        for (int k = 0; k < 3 * N; ++k) wrap01(&s[k]);
        *step += 1;
        forces_impl(P, seed, chain_len, box, N, n_chains, s, c, h, L0, (uint32_t)*step, F, W, err, mode, NULL, hc);
        for (int k = 0; k < 3 * N; ++k) c[k] += 0.5 * dt * F[k] / m;
        afbc_relax(P, seed, box, st, 1, N, s, c, h, G, hc, hb, zeta);
        double K[6] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < N; ++i) {
            double x = h[0] * (s[3 * i] - 0.5) + h[1] * (s[3 * i + 1] - 0.5);
            double y = h[3] * (s[3 * i] - 0.5) + h[4] * (s[3 * i + 1] - 0.5);
            if (oracle_afbc_region(x, y, hc, hb) != 0) continue;
            double dv[3] = {c[3 * i] - (G[0] * x + G[1] * y), c[3 * i + 1] - (G[3] * x + G[4] * y), c[3 * i + 2]};
            for (int q6 = 0; q6 < 6; ++q6) K[q6] += m * dv[SI[q6]] * dv[SJ[q6]];
        }
        for (int q6 = 0; q6 < 6; ++q6) {
            double tot = K[q6] + W[q6] + W[6 + q6] + W[12 + q6] + W[18 + q6];
            if (!isfinite(tot / Vc)) *err |= ORACLE_ERR_NONFINITE;
            acc[q6] += -K[q6] / Vc;
            for (int part = 0; part < 4; ++part) acc[6 * (part + 1) + q6] += -W[6 * part + q6] / Vc;
        }
    }
    for (int q6 = 0; q6 < 6; ++q6) {
        double tot = 0.0;
        for (int part = 0; part < 5; ++part) tot += acc[6 * part + q6];
        if (stress_mean) stress_mean[q6] = tot / nsteps;
    }
    if (parts_mean)
        for (int k = 0; k < 30; ++k) parts_mean[k] = acc[k] / nsteps;
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
