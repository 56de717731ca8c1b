// lhmm_sph.hip -- gfx950 kernels and runtime of the SPH macro side and of the
// coupled exchange interval (include/lhmm.h, lhmm_sph_* and
// lhmm_couple_step).
//
// The macro problem is small (10^3-10^4 particles) and double precision:
// each kernel gives one wave per particle I; lane l takes candidates l,
// l + 64, ... of a fixed enumeration (the particles of the 3 x 3 cells of
// side >= h around I, cell by cell and by index inside a cell; every
// particle when the periodic box holds fewer than 3 cells per side) with the
// minimum image of the periodic box, and a fixed shuffle tree adds the 64
// partial sums, so every sum has a fixed order.  The cells are rebuilt by a
// one-workgroup counting sort before every density pass.  A step is
//   k_density -> k_accel -> k_kick_drift -> k_density -> k_accel -> k_kick
//   -> k_gradL
// (velocity-Verlet, then the micro-domain gradients at the new state).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "lhmm.h"
#include "lhmm_internal.h"

namespace {

constexpr int TPB = 256;             // threads per block
constexpr int WPB = TPB / 64;        // particles (waves) per block

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double pow4(double x) {
    const double x2 = x * x;
    return x2 * x2;
}

struct SphCtx {
    int n, n_mobile, force_mode;  // particles n_mobile .. n-1 are frozen walls
    int kernel;                   // LHMM_KERNEL_QUINTIC or LHMM_KERNEL_LUCY
    int micro_dim;                // 3: micro-domains are 3-D boxes; 2: planar cells (no zz stress)
    int ncx, ncy;                 // cell grid (0: all pairs)
    int* cstart;                  // ncx * ncy + 1 cell offsets into cidx
    int* cidx;                    // particle indices in cell order
    double rho0, eta, zeta, c, theta, F, h, dt, mass, Lx, Ly, lambda_star, alpha;
    double* r;    // n x 2
    double* v;    // n x 2
    double* d;    // n
    double* p;    // n
    double* acc;  // n x 2
};

// quintic kernel of support radius h, q = 3 r / h
__device__ __forceinline__ double quintic_W(double r, double h) {
    const double q = 3.0 * r / h;
    if (q >= 3.0) return 0.0;
    double w = pow4(3.0 - q) * (3.0 - q);
    if (q < 2.0) w -= 6.0 * pow4(2.0 - q) * (2.0 - q);
    if (q < 1.0) w += 15.0 * pow4(1.0 - q) * (1.0 - q);
    return 63.0 / (478.0 * M_PI * h * h) * w;
}

// F = -W'(r) / r
__device__ __forceinline__ double quintic_F(double r, double h) {
    const double q = 3.0 * r / h;
    if (q >= 3.0) return 0.0;
    double dw = -5.0 * pow4(3.0 - q);
    if (q < 2.0) dw += 30.0 * pow4(2.0 - q);
    if (q < 1.0) dw -= 75.0 * pow4(1.0 - q);
    return -(63.0 / (478.0 * M_PI * h * h) * dw * 3.0 / h) / r;
}

// 2-D Lucy kernel, Eq. (lucy_kernel): W = 5/(pi h^2) (1 + 3q)(1 - q)^3, q = r/h
__device__ __forceinline__ double lucy_W(double r, double h) {
    const double q = r / h;
    if (q >= 1.0) return 0.0;
    const double u = 1.0 - q;
    return 5.0 / (M_PI * h * h) * (1.0 + 3.0 * q) * (u * u * u);
}

// its -W'(r)/r reduces to 60 (1 - q)^2 / (pi h^4)
__device__ __forceinline__ double lucy_F(double r, double h) {
    const double q = r / h;
    if (q >= 1.0) return 0.0;
    const double u = 1.0 - q, h2 = h * h;
    return 60.0 / (M_PI * h2 * h2) * (u * u);
}

// the kernel choice is one value per engine, so the branch is uniform
__device__ __forceinline__ double kernel_W(const SphCtx& S, double r) {
    return S.kernel == LHMM_KERNEL_LUCY ? lucy_W(r, S.h) : quintic_W(r, S.h);
}

__device__ __forceinline__ double kernel_F(const SphCtx& S, double r) {
    return S.kernel == LHMM_KERNEL_LUCY ? lucy_F(r, S.h) : quintic_F(r, S.h);
}

__device__ __forceinline__ void min_image(const SphCtx& S, double& dx, double& dy) {
    dx -= S.Lx * rint(dx / S.Lx);
    dy -= S.Ly * rint(dy / S.Ly);
}

__device__ __forceinline__ int cell_x(const SphCtx& S, double x) {
    return min(max((int)(x * (double)S.ncx / S.Lx), 0), S.ncx - 1);
}
__device__ __forceinline__ int cell_y(const SphCtx& S, double y) {
    return min(max((int)(y * (double)S.ncy / S.Ly), 0), S.ncy - 1);
}

// The candidates of a particle at (x, y) in their fixed enumeration.
struct Nbr {
    int total;
    int base[9], pre[10];
    const int* cidx;
    int cells;
    __device__ int get(int t) const {
        if (!cells) return t;
        int k = 0;
        while (t >= pre[k + 1]) ++k;
        return cidx[base[k] + t - pre[k]];
    }
};

__device__ __forceinline__ Nbr neighbours(const SphCtx& S, double x, double y) {
    Nbr nb;
    nb.cidx = S.cidx;
    nb.cells = S.ncx > 0;
    if (!nb.cells) {
        nb.total = S.n;
        return nb;
    }
    const int cx = cell_x(S, x), cy = cell_y(S, y);
    int acc = 0;
    for (int k = 0; k < 9; ++k) {
        const int ax = (cx + k / 3 - 1 + S.ncx) % S.ncx, ay = (cy + k % 3 - 1 + S.ncy) % S.ncy;
        const int c = ax * S.ncy + ay;
        nb.pre[k] = acc;
        nb.base[k] = S.cstart[c];
        acc += S.cstart[c + 1] - S.cstart[c];
    }
    nb.pre[9] = acc;
    nb.total = acc;
    return nb;
}

// Counting sort of all particles into the cell grid, one workgroup; indices
// sorted inside every cell.  Dynamic LDS: ncx * ncy counters + n indices.
__global__ __launch_bounds__(1024) void k_sph_bin(SphCtx S) {
    extern __shared__ int lds[];
    __shared__ int wsum[16];
    const int ncell = S.ncx * S.ncy;
    int* cnt = lds;
    int* lidx = lds + ncell;
    for (int k = threadIdx.x; k < ncell; k += 1024) cnt[k] = 0;
    __syncthreads();
    for (int I = threadIdx.x; I < S.n; I += 1024)
        atomicAdd(&cnt[cell_x(S, S.r[2 * I]) * S.ncy + cell_y(S, S.r[2 * I + 1])], 1);
    __syncthreads();
    int carry = 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int base = 0; base < ncell; base += 1024) {
        const int k = base + (int)threadIdx.x;
        const int v = k < ncell ? cnt[k] : 0;
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wv) before += wsum[w];
            total += wsum[w];
        }
        const int excl = carry + before + x - v;
        __syncthreads();
        if (k < ncell) {
            S.cstart[k] = excl;
            cnt[k] = excl;
        }
        carry += total;
    }
    if (threadIdx.x == 0) S.cstart[ncell] = carry;
    __syncthreads();
    for (int I = threadIdx.x; I < S.n; I += 1024)
        lidx[atomicAdd(&cnt[cell_x(S, S.r[2 * I]) * S.ncy + cell_y(S, S.r[2 * I + 1])], 1)] = I;
    __syncthreads();
    for (int k = threadIdx.x; k < ncell; k += 1024) {
        const int q0 = k == 0 ? 0 : cnt[k - 1], q1 = cnt[k];
        for (int q = q0 + 1; q < q1; ++q) {
            const int key = lidx[q];
            int r = q - 1;
            while (r >= q0 && lidx[r] > key) {
                lidx[r + 1] = lidx[r];
                --r;
            }
            lidx[r + 1] = key;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.n; q += 1024) S.cidx[q] = lidx[q];
}

__global__ __launch_bounds__(TPB) void k_density(SphCtx S) {
    const int I = blockIdx.x * WPB + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (I >= S.n) return;  // wave-uniform
    const double xi = S.r[2 * I], yi = S.r[2 * I + 1];
    const Nbr nb = neighbours(S, xi, yi);
    double s = 0.0;
    for (int t = lane; t < nb.total; t += 64) {
        const int J = nb.get(t);
        double dx = xi - S.r[2 * J], dy = yi - S.r[2 * J + 1];
        min_image(S, dx, dy);
        s += kernel_W(S, sqrt(dx * dx + dy * dy));
    }
    s = wave_sum(s);
    if (lane == 0) {
        S.d[I] = s;
        const double B = S.c * S.c * S.rho0 / 7.0;
        const double x = S.mass * s / S.rho0, x2 = x * x;
        S.p[I] = B * (x2 * x2 * x2 * x - 1.0) + S.theta * B;
    }
}

// polymer stress of particle I: alpha/lambda* x in-plane part of the
// deviatoric part of its micro-domain's mean stress (xx, yy, zz, xy, xz,
// yz).  A 3-D micro-domain loses its isotropic part tr/3; a planar one has
// no zz stress (its particles and forces lie in the plane), so its
// deviatoric part is taken in the plane, (xx + yy)/2 off the diagonal.
__device__ __forceinline__ void polymer_stress(const SphCtx& S, const double* sigma, int I, double& xx, double& xy,
                                               double& yy) {
    if (!sigma) {
        xx = xy = yy = 0.0;
        return;
    }
    const double* g = sigma + 6 * I;
    const double s = S.alpha / S.lambda_star;
    const double iso = S.micro_dim == 2 ? 0.5 * (g[0] + g[1]) : (g[0] + g[1] + g[2]) / 3.0;
    xx = s * (g[0] - iso);
    xy = s * g[3];
    yy = s * (g[1] - iso);
}

// Eq. (sph_continuity) divided by the mass, plus the body force
__global__ __launch_bounds__(TPB) void k_accel(SphCtx S, const double* __restrict__ sigma) {
    const int I = blockIdx.x * WPB + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (I >= S.n_mobile) return;  // wave-uniform
    const double av = 2.0 * S.eta - S.zeta, bv = 4.0 * S.zeta + 2.0 * S.eta;
    const double xi = S.r[2 * I], yi = S.r[2 * I + 1], vxi = S.v[2 * I], vyi = S.v[2 * I + 1];
    const double di = S.d[I], pi_ = S.p[I];
    double pxx, pxy, pyy;
    polymer_stress(S, sigma, I, pxx, pxy, pyy);
    const double i2 = 1.0 / (di * di);
    const Nbr nb = neighbours(S, xi, yi);
    double fx = 0.0, fy = 0.0;
    for (int t = lane; t < nb.total; t += 64) {
        const int J = nb.get(t);
        if (J == I) continue;
        double dx = xi - S.r[2 * J], dy = yi - S.r[2 * J + 1];
        min_image(S, dx, dy);
        const double rr = sqrt(dx * dx + dy * dy);
        if (rr >= S.h || rr == 0.0) continue;
        const double F = kernel_F(S, rr);
        const double ex = dx / rr, ey = dy / rr;
        const double vx = vxi - S.v[2 * J], vy = vyi - S.v[2 * J + 1];
        const double dj = S.d[J];
        const double j2 = 1.0 / (dj * dj);
        const bool wall = J >= S.n_mobile;
        const double pp = pi_ * i2 + S.p[J] * j2;
        fx += pp * F * dx;
        fy += pp * F * dy;
        const double ve = vx * ex + vy * ey;
        const double vis = F / (di * dj);
        fx -= (av * vx + bv * ve * ex) * vis;
        fy -= (av * vy + bv * ve * ey) * vis;
        double qxx = 0.0, qxy = 0.0, qyy = 0.0;
        if (!wall) polymer_stress(S, sigma, J, qxx, qxy, qyy);
        const double sxx = pxx * i2 + qxx * j2, sxy = pxy * i2 + qxy * j2, syy = pyy * i2 + qyy * j2;
        fx -= (sxx * dx + sxy * dy) * F;
        fy -= (sxy * dx + syy * dy) * F;
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    if (lane == 0) {
        const double body = (S.force_mode == LHMM_FORCE_UNIFORM || yi >= 0.5 * S.Ly) ? S.F : -S.F;
        S.acc[2 * I] = fx / S.mass + body;
        S.acc[2 * I + 1] = fy / S.mass;
    }
}

__device__ __forceinline__ double wrap_len(double x, double L) {
    x -= L * floor(x / L);
    return x >= L ? 0.0 : x;
}

__global__ void k_kick_drift(SphCtx S) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= S.n_mobile) return;
    const double hdt = 0.5 * S.dt;
    const double vx = S.v[2 * I] + hdt * S.acc[2 * I], vy = S.v[2 * I + 1] + hdt * S.acc[2 * I + 1];
    S.v[2 * I] = vx;
    S.v[2 * I + 1] = vy;
    S.r[2 * I] = wrap_len(S.r[2 * I] + S.dt * vx, S.Lx);
    S.r[2 * I + 1] = wrap_len(S.r[2 * I + 1] + S.dt * vy, S.Ly);
}

__global__ void k_kick(SphCtx S) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= S.n_mobile) return;
    const double hdt = 0.5 * S.dt;
    S.v[2 * I] += hdt * S.acc[2 * I];
    S.v[2 * I + 1] += hdt * S.acc[2 * I + 1];
}

// Eq. (macro_micro) with 1/d_J: G_ab = d_a v_b; micro gradient
// L = lambda* x traceless part of G^T (u = L r), 3x3 row-major, zero z.
__global__ __launch_bounds__(TPB) void k_gradL(SphCtx S, double* __restrict__ gradL) {
    const int I = blockIdx.x * WPB + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (I >= S.n) return;  // wave-uniform
    if (I >= S.n_mobile) {
        if (lane < 9) gradL[9 * I + lane] = 0.0;
        return;
    }
    const double xi = S.r[2 * I], yi = S.r[2 * I + 1], vxi = S.v[2 * I], vyi = S.v[2 * I + 1];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
    const Nbr nb = neighbours(S, xi, yi);
    for (int t = lane; t < nb.total; t += 64) {
        const int J = nb.get(t);
        if (J == I) continue;
        double dx = xi - S.r[2 * J], dy = yi - S.r[2 * J + 1];
        min_image(S, dx, dy);
        const double rr = sqrt(dx * dx + dy * dy);
        if (rr >= S.h || rr == 0.0) continue;
        const double F = kernel_F(S, rr) / S.d[J];
        const double vx = vxi - S.v[2 * J], vy = vyi - S.v[2 * J + 1];
        g0 += F * dx * vx;
        g1 += F * dx * vy;
        g2 += F * dy * vx;
        g3 += F * dy * vy;
    }
    g0 = wave_sum(g0);
    g1 = wave_sum(g1);
    g2 = wave_sum(g2);
    g3 = wave_sum(g3);
    if (lane != 0) return;
    const double half_tr = 0.5 * (g0 + g3);
    double* o = gradL + 9 * I;
    o[0] = S.lambda_star * (g0 - half_tr);
    o[1] = S.lambda_star * g2;
    o[2] = 0.0;
    o[3] = S.lambda_star * g1;
    o[4] = S.lambda_star * (g3 - half_tr);
    o[5] = 0.0;
    o[6] = 0.0;
    o[7] = 0.0;
    o[8] = 0.0;
}

}  // namespace

struct lhmm_sph {
    SphCtx S{};
    hipStream_t stream = nullptr;
    double* d_sigma = nullptr;  // n x 6, micro stresses of the last interval (zero at start)
    double* d_gradL = nullptr;  // n x 9
    void* bufs[9] = {};
};

namespace {

void sph_release(lhmm_sph* s) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void* b : s->bufs)
        if (b) (void)hipFree(b);
}

// cell lists (when the grid is in use) and densities at the current positions
void launch_density(lhmm_sph* s) {
    const int gw = (s->S.n + WPB - 1) / WPB;
    if (s->S.ncx > 0) {
        const size_t bytes = sizeof(int) * ((size_t)s->S.ncx * s->S.ncy + (size_t)s->S.n);
        k_sph_bin<<<1, 1024, bytes, s->stream>>>(s->S);
    }
    k_density<<<gw, TPB, 0, s->stream>>>(s->S);
}

void launch_sph_step(lhmm_sph* s, const double* sigma, double* gradL) {
    const int gw = (s->S.n + WPB - 1) / WPB;  // wave per particle
    const int gt = (s->S.n + TPB - 1) / TPB;  // thread per particle
    hipStream_t st = s->stream;
    launch_density(s);
    k_accel<<<gw, TPB, 0, st>>>(s->S, sigma);
    k_kick_drift<<<gt, TPB, 0, st>>>(s->S);
    launch_density(s);
    k_accel<<<gw, TPB, 0, st>>>(s->S, sigma);
    k_kick<<<gt, TPB, 0, st>>>(s->S);
    if (gradL) k_gradL<<<gw, TPB, 0, st>>>(s->S, gradL);
}

}  // namespace

hipStream_t lhmm_sph_caller_stream(const lhmm_sph* s) { return s->stream; }

void lhmm_sph_counts(const lhmm_sph* s, int* n, int* n_mobile) {
    *n = s->S.n;
    *n_mobile = s->S.n_mobile;
}

extern "C" {

int lhmm_sph_create(const lhmm_sph_params* p, int32_t n, const double* r0, const double* v0, void* stream,
                    lhmm_sph** out) {
    lhmm_clear_error();
    if (!p || !r0 || !v0 || !out) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    *out = nullptr;
    if (n <= 0) return lhmm_fail(LHMM_ERR_ARG, "n must be positive (got %d)", n);
    if (p->n_fixed < 0 || p->n_fixed >= n) return lhmm_fail(LHMM_ERR_ARG, "n_fixed must be in 0..n-1 (got %d)", p->n_fixed);
    if (p->force_mode != LHMM_FORCE_REVERSE && p->force_mode != LHMM_FORCE_UNIFORM)
        return lhmm_fail(LHMM_ERR_ARG, "unknown force_mode %d", p->force_mode);
    if (p->kernel != LHMM_KERNEL_QUINTIC && p->kernel != LHMM_KERNEL_LUCY)
        return lhmm_fail(LHMM_ERR_ARG, "unknown kernel %d", p->kernel);
    if (p->micro_dim != 0 && p->micro_dim != 2 && p->micro_dim != 3)
        return lhmm_fail(LHMM_ERR_ARG, "micro_dim must be 0, 2 or 3 (got %d)", p->micro_dim);
    const double vals[] = {p->rho0, p->eta, p->zeta, p->c, p->theta, p->F, p->h, p->dt, p->mass, p->Lx, p->Ly,
                           p->lambda_star, p->alpha};
    for (double x : vals)
        if (!std::isfinite(x)) return lhmm_fail(LHMM_ERR_ARG, "non-finite SPH parameter");
    if (!(p->rho0 > 0) || !(p->c > 0) || !(p->h > 0) || !(p->dt > 0) || !(p->mass > 0) || !(p->lambda_star > 0) ||
        p->eta < 0 || p->zeta < 0)
        return lhmm_fail(LHMM_ERR_ARG, "SPH parameters out of range");
    if (!(p->Lx > 2 * p->h) || !(p->Ly > 2 * p->h))
        return lhmm_fail(LHMM_ERR_ARG, "the periodic box must be wider than twice the kernel support");
    for (int k = 0; k < 2 * n; ++k) {
        if (!std::isfinite(r0[k]) || !std::isfinite(v0[k])) return lhmm_fail(LHMM_ERR_ARG, "non-finite state");
        const double L = (k % 2 == 0) ? p->Lx : p->Ly;
        if (!(r0[k] >= 0.0 && r0[k] < L)) return lhmm_fail(LHMM_ERR_ARG, "position %d outside the box", k / 2);
    }
    lhmm_sph* s = new (std::nothrow) lhmm_sph();
    if (!s) return lhmm_fail(LHMM_ERR_OOM, "host allocation failed");
    s->stream = (hipStream_t)stream;
    SphCtx& S = s->S;
    S.n = n;
    S.n_mobile = n - p->n_fixed;
    S.force_mode = p->force_mode;
    S.kernel = p->kernel;
    S.micro_dim = p->micro_dim == 2 ? 2 : 3;
    S.rho0 = p->rho0; S.eta = p->eta; S.zeta = p->zeta; S.c = p->c; S.theta = p->theta; S.F = p->F; S.h = p->h;
    S.dt = p->dt; S.mass = p->mass; S.Lx = p->Lx; S.Ly = p->Ly; S.lambda_star = p->lambda_star; S.alpha = p->alpha;
    // cell grid of side >= h: at least 3 x 3 cells, and counters plus indices in 64 KiB of LDS
    {
        const int gx = (int)std::floor(p->Lx / p->h), gy = (int)std::floor(p->Ly / p->h);
        const bool fits = gx >= 3 && gy >= 3 && (long long)gx * gy + n <= (65536 - 64) / 4;
        S.ncx = fits ? gx : 0;
        S.ncy = fits ? gy : 0;
    }
    const size_t sizes[9] = {2 * (size_t)n, 2 * (size_t)n, (size_t)n, (size_t)n, 2 * (size_t)n, 6 * (size_t)n,
                             9 * (size_t)n, (size_t)S.ncx * S.ncy + 1, (size_t)n};
    for (int k = 0; k < 9; ++k) {
        if (hipMalloc(&s->bufs[k], sizes[k] * sizeof(double)) != hipSuccess) {
            sph_release(s);
            delete s;
            return lhmm_fail(LHMM_ERR_OOM, "hipMalloc failed");
        }
    }
    S.r = (double*)s->bufs[0];
    S.v = (double*)s->bufs[1];
    S.d = (double*)s->bufs[2];
    S.p = (double*)s->bufs[3];
    S.acc = (double*)s->bufs[4];
    s->d_sigma = (double*)s->bufs[5];
    s->d_gradL = (double*)s->bufs[6];
    S.cstart = (int*)s->bufs[7];
    S.cidx = (int*)s->bufs[8];
    auto init = [&]() -> int {
        LHMM_HIPCHK(hipMemcpy(S.r, r0, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice));
        LHMM_HIPCHK(hipMemcpy(S.v, v0, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice));
        LHMM_HIPCHK(hipMemset(s->d_sigma, 0, 6 * (size_t)n * sizeof(double)));
        LHMM_HIPCHK(hipMemset(s->d_gradL, 0, 9 * (size_t)n * sizeof(double)));
        return LHMM_OK;
    };
    int rc = init();
    if (rc != LHMM_OK) {
        sph_release(s);
        delete s;
        return rc;
    }
    *out = s;
    return LHMM_OK;
}

int lhmm_sph_step(lhmm_sph* s, const double* sigma, double* gradL_out) {
    lhmm_clear_error();
    if (!s) return lhmm_fail(LHMM_ERR_ARG, "null engine");
    launch_sph_step(s, sigma, gradL_out);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sph_get_state(lhmm_sph* s, double* r, double* v, double* d) {
    lhmm_clear_error();
    if (!s) return lhmm_fail(LHMM_ERR_ARG, "null engine");
    LHMM_HIPCHK(hipStreamSynchronize(s->stream));
    const size_t n = (size_t)s->S.n;
    if (r) LHMM_HIPCHK(hipMemcpy(r, s->S.r, 2 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (v) LHMM_HIPCHK(hipMemcpy(v, s->S.v, 2 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (d) {
        // density at the current positions
        launch_density(s);
        LHMM_HIPCHK(hipGetLastError());
        LHMM_HIPCHK(hipStreamSynchronize(s->stream));
        LHMM_HIPCHK(hipMemcpy(d, s->S.d, n * sizeof(double), hipMemcpyDeviceToHost));
    }
    return LHMM_OK;
}

int lhmm_sph_coupling_state(lhmm_sph* s, double* sigma, double* gradL) {
    lhmm_clear_error();
    if (!s) return lhmm_fail(LHMM_ERR_ARG, "null engine");
    LHMM_HIPCHK(hipStreamSynchronize(s->stream));
    const size_t n = (size_t)s->S.n;
    if (sigma) LHMM_HIPCHK(hipMemcpy(sigma, s->d_sigma, 6 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (gradL) LHMM_HIPCHK(hipMemcpy(gradL, s->d_gradL, 9 * n * sizeof(double), hipMemcpyDeviceToHost));
    return LHMM_OK;
}

int lhmm_couple_step(lhmm_sph* s, lhmm_micro* m, int32_t m_bar, int32_t k_micro) {
    lhmm_clear_error();
    if (!s || !m) return lhmm_fail(LHMM_ERR_ARG, "null engine");
    if (m_bar <= 0) return lhmm_fail(LHMM_ERR_ARG, "m_bar must be positive (got %d)", m_bar);
    if (k_micro <= 0) return lhmm_fail(LHMM_ERR_ARG, "k_micro must be positive (got %d)", k_micro);
    int32_t nb = 0;
    int rc = lhmm_micro_sizes(m, nullptr, &nb);
    if (rc != LHMM_OK) return rc;
    if (nb != s->S.n_mobile)
        return lhmm_fail(LHMM_ERR_ARG, "micro engine holds %d boxes for %d mobile SPH particles", nb, s->S.n_mobile);
    if (lhmm_micro_caller_stream(m) != s->stream)
        return lhmm_fail(LHMM_ERR_ARG, "the SPH and micro engines must share one stream");
    // m_bar SPH steps under the stored micro stresses; the gradient of the
    // last one drives the micro-domains
    for (int k = 0; k < m_bar; ++k) launch_sph_step(s, s->d_sigma, k + 1 == m_bar ? s->d_gradL : nullptr);
    LHMM_HIPCHK(hipGetLastError());
    return lhmm_micro_step(m, s->d_gradL, k_micro, s->d_sigma);
}

int lhmm_sph_destroy(lhmm_sph* s) {
    lhmm_clear_error();
    if (!s) return LHMM_OK;
    sph_release(s);
    delete s;
    return LHMM_OK;
}

}  // extern "C"
