// lhmm_micro.hip -- gfx950 kernels and runtime of the batched micro-DPD
// engine behind include/lhmm.h.
//
// One step of every box (velocity-Verlet of the micro-scale equation of
// motion, Eq. motion, in a periodic cell deformed by the box's velocity
// gradient; Appendix "Detailed Coupling Protocol", Step 3) is three launches
// over a flattened index of all boxes (five with unfused binning):
//   k_bin_box      one workgroup per box: the cell step (FP64: mid-step
//                  cell inverse, deformation h <- exp(L dt) h,
//                  Lagrange-Gauss reduction of the in-plane basis, cell
//                  grid, width guard), the half kick c += dt/2 (F/m - L c)
//                  and drift of the fractional coordinates with the
//                  mid-step cell (remap by the reduction, wrap, cell index),
//                  then a counting sort of the particles by cell in LDS with
//                  each cell sorted by id so every sum has a fixed order
//                  (k_cell_step and k_kick_drift run the first two parts as
//                  separate launches when binning is not fused);
//   k_forces       per particle: conservative + dissipative + random pair
//                  forces (Eqs. conservative, dissipative, random) over the
//                  neighbour cells, FENE springs (Eq. fene_force), the
//                  second half kick with the final force, and the block's
//                  virial and kinetic partial sums in FP64;
//   k_box_stress   one wave per box: virial stress of the step (Eqs.
//                  IKtotal, kinetic_stress, potential_stress with a uniform
//                  weight over the cell), accumulated over the call.
// A box may instead be a micro-domain with boundary regions (Sec.
// "Macro-to-Micro Coupling", Tab. 2): its cell stays fixed, the particles of
// the boundary-condition ring relax toward the imposed field v' = G r' of
// Eq. micro_bc after each half kick (an Ornstein-Uhlenbeck step with thermal
// noise), and its stress is the Irving-Kirkwood stress of the core (kinetic
// part over the core's particles relative to the imposed field, each pair's
// virial weighted by the fraction of its segment inside the core).
// The per-particle kernels run over work blocks of BS particles; a block
// never straddles two boxes, so per-box quantities are uniform in a block
// and reductions stay deterministic.  The step loop is captured in HIP
// graphs.  Particle state is single or double precision (template
// parameter); cells, gradients and stress sums are always double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lhmm.h"
#include "lhmm_internal.h"

namespace {

constexpr int BS = 256;                 // particles per work block
constexpr int BIN_THREADS_MAX = 1024;   // largest binning workgroup (256, 512 or 1024 threads)
constexpr int MAX_CELLS_PER_BOX = 17424;  // binning LDS: cell starts and three per-column offsets (136 KiB)
constexpr int GRAPH_CHUNK = 50;         // default steps per captured graph
constexpr int MAX_GROUPS = 4;           // overlapped box groups of a captured step
constexpr int ACC = 36;                 // per-box stress sums: kinetic, pair, FENE, C, D, R (6 each)

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(LHMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct BoxInfo {
    int off;       // first particle (global index)
    int n;         // particles
    int n_beads;   // n_chains * chain_len
    int cell_off;  // first slot in cell_start (cap + 1 slots per box)
    int cell_cap;  // cell capacity
    int gcell_off; // first slot in gcell_start (2 cap + 1 slots per box)
    int zsub;      // cells per cutoff along z (1 or 2): the z range of a stencil row is 2 zsub + 1 cells
    int blk_off;   // first work block
    int nblk;      // work blocks
    unsigned rng_id;  // box word of the random-force counter
};

struct BoxDyn {  // per-box FP64 state, rewritten every step
    double h[9];
    double L[9];
    double E[9];
    double Eh[9];
    double hmi[9];  // inverse of the mid-step cell
    double vol;
    int U[4];       // in-plane reduction of this step, h_new = h U
    int nc[3];      // cell grid of this step
    int changed;
    // boundary regions (hc > 0): core |x'|, |y'| < hc, ring hc <= max(|x'|, |y'|)
    // < hb, positions relative to the cell centre; G: the imposed in-plane
    // gradient (xx, xy, yx, yy), while the cell's own L stays zero
    double hc, hb;
    double G[4];
};

struct Ctx {
    int n_total, n_boxes, n_blocks, chain_len;
    const BoxInfo* box;
    BoxDyn* dyn;
    unsigned* flags;
    const int* blk_box;
    const int* blk_first;
    // selection: when sel is set, per-box kernels run over the n_sel boxes
    // sel[0..n_sel) and per-block kernels over the work blocks blk_list[..]
    const int* sel;
    const int* blk_list;
    int n_sel;
    void* s;  // SoA: component k of particle i at [k * n_total + i]
    void* c;
    void* f;
    int* pcell;
    int* cell_start;
    // per box, cell-sorted pairs of records: (x, y, z, local index), r = h s,
    // then (cx, cy, cz, local index), 2 x 4 reals per particle (one scattered
    // 32-byte store in the binning, one 32-byte segment per neighbour in the
    // force kernel's evaluation)
    void* cell_pv;
    // Search layout: per box (at 2 x its particle offset) every cell column
    // (m0, m1) as [images of its top zsub cells shifted by -h_z][its cells]
    // [images of its bottom zsub cells shifted by +h_z], so the z cells
    // k2 - zsub .. k2 + zsub around any cell are one contiguous range;
    // gcell_start holds the range starts of these n0 n1 (n2 + 2 zsub) cells.
    // srec: (x, y, z, cell-order position << 5 | 9 x z image: 0 none,
    // 1 below, 2 above), r = h s; padded by four records.
    int* gcell_start;
    void* srec;
    double* part_vir;   // n_blocks x pv_stride: pair virial, FENE virial (+ C, D, R parts)
    int pv_stride;      // 12, or 30 when the conservative, dissipative and random parts are kept
    double vir_scale;   // 1 when each pair is evaluated once, 1/2 when twice
    double* part_kin;   // n_blocks x 6
    unsigned* part_pairs;  // n_blocks: ordered pairs within the cutoff
    double* acc;        // n_boxes x ACC: kinetic, pair, FENE, C, D, R stress sums
    unsigned long long* acc_pairs;  // n_boxes
    unsigned long long* tot_pairs;  // n_boxes, every step since the engine was created
    unsigned long long* step;       // completed steps
    double a, gamma, sigma, rdt, dt, mass, inv_mass, rc, rc2, H, inv_R02;
    double ou_damp, ou_amp;  // ring relaxation over half a step: exp(-zeta dt/2), sqrt(kBT/m (1 - exp(-zeta dt)))
    unsigned key0, key1;
};

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed
// by the seed, counter (min id, max id, step, box); a Box-Muller normal from
// the top 23 bits of the first two output words.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x32_10(unsigned& x0, unsigned& x1, unsigned& x2, unsigned& x3,
                                              unsigned k0, unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * x0;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * x2;
        // three-input xors as one v_bitop3_b32 each (truth table 0x96)
        const unsigned y0 = __builtin_amdgcn_bitop3_b32((unsigned)(p1 >> 32), x1, k0, 0x96);
        const unsigned y2 = __builtin_amdgcn_bitop3_b32((unsigned)(p0 >> 32), x3, k1, 0x96);
        x1 = (unsigned)p1;
        x3 = (unsigned)p0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The pair stream's generator: counter (x0, x1, step, box), where step,
// box and the key are the same for a whole workgroup.  In the first two
// rounds two of the three inputs of one or both xors are then uniform; the
// xors are grouped so that the scalar unit combines those two (one vector
// xor, where a v_bitop3_b32 would need one of them moved to a vector
// register first).  The output equals philox4x32_10's.
__device__ __forceinline__ void philox_pair(unsigned& x0, unsigned& x1, unsigned step, unsigned box, unsigned k0,
                                            unsigned k1) {
    // round 1: M1 step and key are uniform, and so are box and key
    unsigned long long p0 = (unsigned long long)0xD2511F53u * x0;
    unsigned long long p1 = (unsigned long long)0xCD9E8D57u * step;
    unsigned y0 = ((unsigned)(p1 >> 32) ^ k0) ^ x1;
    unsigned y2 = (box ^ k1) ^ (unsigned)(p0 >> 32);
    const unsigned u1 = (unsigned)p1;  // the second word is uniform after round 1
    unsigned x3 = (unsigned)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 2: the second word and key are uniform
    p0 = (unsigned long long)0xD2511F53u * y0;
    p1 = (unsigned long long)0xCD9E8D57u * y2;
    x0 = (u1 ^ k0) ^ (unsigned)(p1 >> 32);
    unsigned x2 = __builtin_amdgcn_bitop3_b32((unsigned)(p0 >> 32), x3, k1, 0x96);
    x1 = (unsigned)p1;
    x3 = (unsigned)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        p0 = (unsigned long long)0xD2511F53u * x0;
        p1 = (unsigned long long)0xCD9E8D57u * x2;
        const unsigned z0 = __builtin_amdgcn_bitop3_b32((unsigned)(p1 >> 32), x1, k0, 0x96);
        const unsigned z2 = __builtin_amdgcn_bitop3_b32((unsigned)(p0 >> 32), x3, k1, 0x96);
        x1 = (unsigned)p1;
        x3 = (unsigned)p0;
        x0 = z0;
        x2 = z2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

template <typename real>
__device__ __forceinline__ real box_muller(unsigned w0, unsigned w1);

// (m + 1/2) 2^-23 for the top 23 bits m of w: the float 1 + m 2^-23 (exponent
// bits 0x7F above m, one funnel shift) less 1 - 2^-24, a subtraction without
// rounding since both lie in [1/2, 2)
__device__ __forceinline__ float unit_open(unsigned w) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)) - 0x1.fffffep-1f;
}

template <>
__device__ __forceinline__ float box_muller<float>(unsigned w0, unsigned w1) {
    const float u0 = unit_open(w0);
    const float u1 = unit_open(w1);
    // v_log_f32 is log2; v_cos_f32 takes its argument in revolutions
    // -2 ln u0 lies in [1e-7, 35]: the hardware square root (1 ulp) needs no range handling
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));  // -2 ln u0
    return r * __builtin_amdgcn_cosf(u1);
}

template <>
__device__ __forceinline__ double box_muller<double>(unsigned w0, unsigned w1) {
    const double u0 = ((double)(w0 >> 9) + 0.5) * 1.1920928955078125e-07;
    const double u1 = ((double)(w1 >> 9) + 0.5) * 1.1920928955078125e-07;
    return sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
}

// both Box-Muller normals (cosine and sine branches) of two output words
template <typename real>
__device__ __forceinline__ void box_muller2(unsigned w0, unsigned w1, real& x, real& y);

template <>
__device__ __forceinline__ void box_muller2<float>(unsigned w0, unsigned w1, float& x, float& y) {
    const float u0 = ((float)(w0 >> 9) + 0.5f) * 1.1920928955078125e-07f;
    const float u1 = ((float)(w1 >> 9) + 0.5f) * 1.1920928955078125e-07f;
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
    x = r * __builtin_amdgcn_cosf(u1);
    y = r * __builtin_amdgcn_sinf(u1);
}

template <>
__device__ __forceinline__ void box_muller2<double>(unsigned w0, unsigned w1, double& x, double& y) {
    const double u0 = ((double)(w0 >> 9) + 0.5) * 1.1920928955078125e-07;
    const double u1 = ((double)(w1 >> 9) + 0.5) * 1.1920928955078125e-07;
    const double r = sqrt(-2.0 * log(u0));
    x = r * cos(2.0 * M_PI * u1);
    y = r * sin(2.0 * M_PI * u1);
}

template <typename real>
__device__ __forceinline__ real pair_theta(unsigned id_i, unsigned id_j, unsigned step, unsigned box,
                                           unsigned k0, unsigned k1) {
    unsigned x0 = min(id_i, id_j), x1 = max(id_i, id_j);
    philox_pair(x0, x1, step, box, k0, k1);
    return box_muller<real>(x0, x1);
}

// ---------------------------------------------------------------------------
// Cell-sorted particle records: (x, y, z, local index) in one 4-vector
// ---------------------------------------------------------------------------

template <typename real>
struct Rec;
template <>
struct Rec<float> {
    using T = float4;
    __device__ static T make(float x, float y, float z, int id) { return make_float4(x, y, z, __int_as_float(id)); }
    __device__ static int id(T v) { return __float_as_int(v.w); }
};
template <>
struct Rec<double> {
    using T = double4;
    __device__ static T make(double x, double y, double z, int id) { return make_double4(x, y, z, (double)id); }
    __device__ static int id(T v) { return (int)v.w; }
};

// Raw buffer view of a record array (stride 0, no range limit in practice):
// a float record is read by one 16-byte buffer load, which the compiler keeps
// whole, so the loads of a search step are issued together and none is
// deferred into the branch that queues a neighbour.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rec_rsrc(const char* base) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
}

template <typename real>
__device__ __forceinline__ typename Rec<real>::T load_rec(__amdgpu_buffer_rsrc_t r, const char* base, unsigned off);

template <>
__device__ __forceinline__ float4 load_rec<float>(__amdgpu_buffer_rsrc_t r, const char*, unsigned off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_float4(__uint_as_float(x.x), __uint_as_float(x.y), __uint_as_float(x.z), __uint_as_float(x.w));
}

template <>
__device__ __forceinline__ double4 load_rec<double>(__amdgpu_buffer_rsrc_t, const char* base, unsigned off) {
    return *(const double4*)(base + off);
}

// ---------------------------------------------------------------------------
// FP64 cell algebra (row-major 3x3; columns are lattice vectors)
// ---------------------------------------------------------------------------

__host__ __device__ inline void m3_mul(const double* A, const double* B, double* C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    for (int k = 0; k < 9; ++k) C[k] = T[k];
}

__host__ __device__ inline double m3_det(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

__host__ __device__ inline void m3_inv(const double* A, double* B) {
    const double id = 1.0 / m3_det(A);
    double T[9];
    T[0] = (A[4] * A[8] - A[5] * A[7]) * id;
    T[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    T[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    T[3] = (A[5] * A[6] - A[3] * A[8]) * id;
    T[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    T[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    T[6] = (A[3] * A[7] - A[4] * A[6]) * id;
    T[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    T[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    for (int k = 0; k < 9; ++k) B[k] = T[k];
}

// perpendicular widths w_a = V / |h_b x h_c|
__host__ __device__ inline void m3_widths(const double* h, double* w) {
    const double V = fabs(m3_det(h));
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const double ux = h[b], uy = h[3 + b], uz = h[6 + b];
        const double vx = h[c], vy = h[3 + c], vz = h[6 + c];
        const double x = uy * vz - uz * vy, y = uz * vx - ux * vz, z = ux * vy - uy * vx;
        w[a] = V / sqrt(x * x + y * y + z * z);
    }
}

// Is L finite, in-plane and traceless?
__host__ __device__ inline bool gradient_ok(const double* L) {
    double scale = 1.0;
    for (int k = 0; k < 9; ++k) {
        if (!(fabs(L[k]) <= 1e300)) return false;
        scale += fabs(L[k]);
    }
    if (L[2] != 0.0 || L[5] != 0.0 || L[6] != 0.0 || L[7] != 0.0 || L[8] != 0.0) return false;
    return fabs(L[0] + L[4]) <= 1e-12 * scale;
}

// exp(L tau) for in-plane traceless L: in the plane L^2 = k^2 I, k^2 = a^2 + bc,
// so exp(L tau) = f0 I + f1 L with (cosh, sinh/k), (cos, sin/w) or (1, tau).
__host__ __device__ inline void expm_planar(const double* L, double tau, double* E) {
    const double a = 0.5 * (L[0] - L[4]), b = L[1], c = L[3];
    const double k2 = a * a + b * c;
    double f0, f1;
    if (k2 > 0.0) {
        const double k = sqrt(k2);
        f0 = cosh(k * tau);
        f1 = sinh(k * tau) / k;
    } else if (k2 < 0.0) {
        const double w = sqrt(-k2);
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

// Lagrange-Gauss reduction of the in-plane basis (columns 0 and 1 of h);
// swaps as (b1, b2) -> (b2, -b1), size reductions b2 -= m b1 with
// m = floor(mu + 1/2).  U accumulates h_new = h U (det U = +1).
__host__ __device__ inline int reduce_planar(double* h, int* U) {
    double b1x = h[0], b1y = h[3], b2x = h[1], b2y = h[4];
    long long u00 = 1, u01 = 0, u10 = 0, u11 = 1;
    int changed = 0;
    for (int it = 0; it < 256; ++it) {
        const double n1 = b1x * b1x + b1y * b1y, n2 = b2x * b2x + b2y * b2y;
        if (n2 < n1) {
            const double tx = b1x, ty = b1y;
            b1x = b2x; b1y = b2y;
            b2x = -tx; b2y = -ty;
            const long long a0 = u01, a1 = -u00, c0 = u11, c1 = -u10;
            u00 = a0; u01 = a1; u10 = c0; u11 = c1;
            changed = 1;
            continue;
        }
        const long long m = (long long)floor((b1x * b2x + b1y * b2y) / n1 + 0.5);
        if (m == 0) break;
        b2x -= (double)m * b1x;
        b2y -= (double)m * b1y;
        u01 -= m * u00;
        u11 -= m * u10;
        changed = 1;
    }
    h[0] = b1x; h[3] = b1y; h[1] = b2x; h[4] = b2y;
    U[0] = (int)u00; U[1] = (int)u01; U[2] = (int)u10; U[3] = (int)u11;
    return changed;
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

// Sum NV doubles over the workgroup (BS threads); thread 0 returns the sums.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* NV * (BS/64) */) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wv * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = 0.0;
            for (int w = 0; w < BS / 64; ++w) t += sh[w * NV + k];
            v[k] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

constexpr int N_XCD = 8;  // MI355X: workgroups are dealt to the 8 XCDs round robin

// Work item of workgroup b out of n, chosen so that each XCD (b mod 8) gets
// one contiguous run of work items: the blocks of a box then share one L2.
__device__ __forceinline__ int xcd_local_work(int b, int n) {
    const int x = b % N_XCD, l = b / N_XCD;
    const int per = n / N_XCD, rem = n % N_XCD;
    return x * per + min(x, rem) + l;
}

// Per call: take each box's gradient (device array n_boxes x 9), validate,
// and form exp(L dt), exp(L dt/2).
__global__ void k_setup_call(Ctx C, const double* __restrict__ gradL) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= C.n_boxes) return;
    BoxDyn& D = C.dyn[b];
    double L[9];
    for (int k = 0; k < 9; ++k) L[k] = gradL[9 * b + k];
    if (!gradient_ok(L)) {
        for (int k = 0; k < 9; ++k) L[k] = 0.0;
        C.flags[b] |= LHMM_FLAG_ARG;
    }
    if (D.hc > 0.0) {  // boundary regions: the gradient drives the ring, the cell stays fixed
        D.G[0] = L[0]; D.G[1] = L[1]; D.G[2] = L[3]; D.G[3] = L[4];
        for (int k = 0; k < 9; ++k) L[k] = 0.0;
    }
    for (int k = 0; k < 9; ++k) D.L[k] = L[k];
    expm_planar(L, C.dt, D.E);
    expm_planar(L, 0.5 * C.dt, D.Eh);
}

// Remove each box's mean peculiar velocity (one workgroup per box, or per
// selected box).  The pair forces cancel, so the mean obeys
// d<c>/dt = -L <c>: a flow that compresses the box amplifies it, and the
// rounding of the two-sided single-precision pair forces seeds it.  The
// micro-domain moves with its macro particle, so its mean is zero.
template <typename real>
__global__ __launch_bounds__(256) void k_remove_mean(Ctx C) {
    const int b = C.sel ? C.sel[blockIdx.x] : blockIdx.x;
    const BoxInfo B = C.box[b];
    const int N = C.n_total;
    real* c = (real*)C.c;
    __shared__ double red[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    // thread t adds particles t, t + 256, ... in that order; four particles'
    // loads are issued before their additions
    const real* cb = c + B.off;
    int i = threadIdx.x;
    for (; i + 3 * 256 < B.n; i += 4 * 256) {
        real v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) v[u][k] = cb[(long)k * N + i + u * 256];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k] += (double)v[u][k];
    }
    for (; i < B.n; i += 256)
        for (int k = 0; k < 3; ++k) acc[k] += (double)cb[(long)k * N + i];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    const real mean[3] = {(real)(red[0][0] / B.n), (real)(red[1][0] / B.n), (real)(red[2][0] / B.n)};
    real* cw = c + B.off;
#pragma unroll 4
    for (int j = threadIdx.x; j < B.n; j += 256)
        for (int k = 0; k < 3; ++k) cw[(long)k * N + j] -= mean[k];
}

__global__ void k_zero_acc(Ctx C) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ACC * C.n_boxes) C.acc[t] = 0.0;
    if (t < C.n_boxes) C.acc_pairs[t] = 0ull;
}

// One thread per box.  advance = 1: mid-step inverse, deformation and
// reduction of this step; advance = 0: grid for the current cell only.
__device__ void cell_step_box(const Ctx& C, int b, int advance);

__global__ void k_cell_step(Ctx C, int advance) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (C.sel ? C.n_sel : C.n_boxes)) return;
    cell_step_box(C, C.sel ? C.sel[q] : q, advance);
}

__device__ void cell_step_box(const Ctx& C, int b, int advance) {
    BoxDyn& D = C.dyn[b];
    double h[9];
    for (int k = 0; k < 9; ++k) h[k] = D.h[k];
    int U[4] = {1, 0, 0, 1};
    int changed = 0;
    if (advance) {
        double hm[9];
        m3_mul(D.Eh, h, hm);
        m3_inv(hm, D.hmi);
        m3_mul(D.E, h, h);
        changed = reduce_planar(h, U);
        for (int k = 0; k < 9; ++k) D.h[k] = h[k];
    }
    for (int k = 0; k < 4; ++k) D.U[k] = U[k];
    D.changed = changed;
    // the stress is averaged over the core of a boundary-region box
    D.vol = D.hc > 0.0 ? 4.0 * D.hc * D.hc * h[8] : fabs(m3_det(h));
    double w[3];
    m3_widths(h, w);
    int nc[3];
    bool narrow = false;
    const int zsub = C.box[b].zsub, zmin = 2 * zsub + 1;
    for (int a = 0; a < 3; ++a) {
        const int sub = a == 2 ? zsub : 1;
        int n = (int)floor(sub * w[a] / C.rc);
        if (!(w[a] >= 3.0 * C.rc)) narrow = true;
        if (n < 2 * sub + 1) n = 2 * sub + 1;
        nc[a] = n;
    }
    const int cap = C.box[b].cell_cap;
    while ((long long)nc[0] * nc[1] * nc[2] > cap) {  // only reachable for a flagged (narrow) cell
        int a = nc[0] >= nc[1] ? 0 : 1;
        if (nc[a] <= 3) {
            if (nc[2] <= zmin) break;
            a = 2;
        }
        nc[a] -= 1;
    }
    if (narrow) C.flags[b] |= LHMM_FLAG_CELL;
    if (!(fmin(fmin(w[0], w[1]), w[2]) >= LHMM_THIN_WIDTH * C.rc)) C.flags[b] |= LHMM_FLAG_THIN;
    D.nc[0] = nc[0]; D.nc[1] = nc[1]; D.nc[2] = nc[2];
}

template <typename real>
__device__ __forceinline__ void cell_coords(real s0, real s1, real s2, const int* nc, int& k0, int& k1, int& k2) {
    k0 = min(max((int)(s0 * (real)nc[0]), 0), nc[0] - 1);
    k1 = min(max((int)(s1 * (real)nc[1]), 0), nc[1] - 1);
    k2 = min(max((int)(s2 * (real)nc[2]), 0), nc[2] - 1);
}

template <typename real>
__device__ __forceinline__ int cell_of(real s0, real s1, real s2, const int* nc) {
    int k0, k1, k2;
    cell_coords(s0, s1, s2, nc, k0, k1, k2);
    return (k0 * nc[1] + k1) * nc[2] + k2;
}

// a / d for 0 <= a < 2^22 and d >= 1, given inv = 1.0f / d: single-precision
// rounding moves (a + 1/2) / d by less than the 1/(2d) it keeps from integers
__device__ __forceinline__ int div_small(int a, float inv) { return (int)(((float)a + 0.5f) * inv); }

template <typename real>
__device__ __forceinline__ real wrap01(real x) {
    x -= floor(x);
    return x >= (real)1 ? (real)0 : x;
}

// The ring of a boundary-region box (Eq. micro_bc): a particle at in-plane
// position (x, y) relative to the cell centre with hc <= max(|x|, |y|) < hb
// has its in-plane velocity relaxed toward the imposed field u = G r' over
// half a step, c <- u + (c - u) damp + amp xi, with the normal pair xi of
// Philox4x32-10 at counter (id, 0xFFFFFFF0 + half, step, box).
template <typename real>
__device__ __forceinline__ void ring_relax(real x, real y, real hc, real hb, const real (&G)[4], real damp, real amp,
                                           unsigned id, unsigned half, unsigned step, unsigned box, unsigned k0,
                                           unsigned k1, real& c0, real& c1) {
    const real mx = fmax(fabs(x), fabs(y));
    if (!(mx >= hc && mx < hb)) return;
    unsigned x0 = id, x1 = 0xFFFFFFF0u + half, x2 = step, x3 = box;
    philox4x32_10(x0, x1, x2, x3, k0, k1);
    real n0, n1;
    box_muller2<real>(x0, x1, n0, n1);
    const real u0 = G[0] * x + G[1] * y, u1 = G[2] * x + G[3] * y;
    c0 = u0 + (c0 - u0) * damp + amp * n0;
    c1 = u1 + (c1 - u1) * damp + amp * n1;
}

// A box's step constants for the half kick and drift, read once into
// registers (the per-particle stores could otherwise force reloads).
template <typename real>
struct KickDrift {
    real hdt, im, dt, L0, L1, L3, L4, M[9];
    int changed, U[4], nc[3];
    // boundary regions: half-widths, imposed gradient, the cell's in-plane
    // basis and random-stream words of the first half kick
    bool afbc;
    real hc, hb, G[4], h00, h01, h10, h11, damp, amp;
    unsigned step, box, k0, k1;
    __device__ explicit KickDrift(const Ctx& C, const BoxDyn& D, unsigned box_rng = 0) {
        hdt = (real)(0.5 * C.dt);
        im = (real)C.inv_mass;
        dt = (real)C.dt;
        L0 = (real)D.L[0]; L1 = (real)D.L[1]; L3 = (real)D.L[3]; L4 = (real)D.L[4];
        for (int k = 0; k < 9; ++k) M[k] = (real)D.hmi[k];
        changed = D.changed;
        for (int k = 0; k < 4; ++k) U[k] = D.U[k];
        for (int k = 0; k < 3; ++k) nc[k] = D.nc[k];
        afbc = D.hc > 0.0;
        hc = (real)D.hc; hb = (real)D.hb;
        for (int k = 0; k < 4; ++k) G[k] = (real)D.G[k];
        h00 = (real)D.h[0]; h01 = (real)D.h[1]; h10 = (real)D.h[3]; h11 = (real)D.h[4];
        damp = (real)C.ou_damp; amp = (real)C.ou_amp;
        step = (unsigned)(*C.step + 1ull);  // the step being made
        box = box_rng; k0 = C.key0; k1 = C.key1;
    }
};

// Half kick c += dt/2 (F/m - L c), drift of the fractional coordinate with
// the mid-step cell, remap after a reduction, wrap (in registers).
template <typename real>
__device__ __forceinline__ void kick_drift(const KickDrift<real>& K, real (&sv)[3], real (&cv)[3], const real (&fv)[3],
                                           int id) {
    // in-plane L: (L c)_z = 0
    const real lc0 = K.L0 * cv[0] + K.L1 * cv[1], lc1 = K.L3 * cv[0] + K.L4 * cv[1];
    cv[0] += K.hdt * (fv[0] * K.im - lc0);
    cv[1] += K.hdt * (fv[1] * K.im - lc1);
    cv[2] += K.hdt * (fv[2] * K.im);
    if (K.afbc) {
        const real x = K.h00 * (sv[0] - (real)0.5) + K.h01 * (sv[1] - (real)0.5);
        const real y = K.h10 * (sv[0] - (real)0.5) + K.h11 * (sv[1] - (real)0.5);
        ring_relax<real>(x, y, K.hc, K.hb, K.G, K.damp, K.amp, (unsigned)id, 0u, K.step, K.box, K.k0, K.k1, cv[0], cv[1]);
    }
    real s0 = sv[0] + K.dt * (K.M[0] * cv[0] + K.M[1] * cv[1] + K.M[2] * cv[2]);
    real s1 = sv[1] + K.dt * (K.M[3] * cv[0] + K.M[4] * cv[1] + K.M[5] * cv[2]);
    const real s2 = sv[2] + K.dt * (K.M[6] * cv[0] + K.M[7] * cv[1] + K.M[8] * cv[2]);
    if (K.changed) {  // s <- U^{-1} s in the plane, U^{-1} = [[u11, -u01], [-u10, u00]]
        const real x = s0, y = s1;
        s0 = (real)K.U[3] * x - (real)K.U[1] * y;
        s1 = -(real)K.U[2] * x + (real)K.U[0] * y;
    }
    sv[0] = wrap01(s0); sv[1] = wrap01(s1); sv[2] = wrap01(s2);
}

// Half kick and drift of particle i (advance = 1) and its cell; returns the
// cell (stored to pcell when store_cell is set).
template <typename real>
__device__ __forceinline__ int kick_drift_particle(const Ctx& C, const KickDrift<real>& K, int i, int local, int advance,
                                                   bool store_cell = true) {
    const int N = C.n_total;
    real* s = (real*)C.s;
    real* c = (real*)C.c;
    const real* f = (const real*)C.f;
    real sv[3] = {s[i], s[N + i], s[2 * N + i]};
    if (advance) {
        real cv[3] = {c[i], c[N + i], c[2 * N + i]};
        const real fv[3] = {f[i], f[N + i], f[2 * N + i]};
        kick_drift<real>(K, sv, cv, fv, local);
        c[i] = cv[0]; c[N + i] = cv[1]; c[2 * N + i] = cv[2];
        s[i] = sv[0]; s[N + i] = sv[1]; s[2 * N + i] = sv[2];
    }
    const int cell = cell_of(sv[0], sv[1], sv[2], K.nc);
    if (store_cell) C.pcell[i] = cell;
    return cell;
}

template <typename real>
__global__ __launch_bounds__(BS) void k_kick_drift(Ctx C, int advance) {
    const int blk = C.blk_list ? C.blk_list[blockIdx.x] : (int)blockIdx.x;
    const int b = C.blk_box[blk];
    const BoxInfo B = C.box[b];
    const int i = C.blk_first[blk] + (int)threadIdx.x;
    if (i >= B.off + B.n) return;
    const KickDrift<real> K(C, C.dyn[b], B.rng_id);
    kick_drift_particle<real>(C, K, i, i - B.off, advance);
}

// Exclusive scan over k in [0, n) of val(k) by a workgroup of BT threads:
// each thread sums a run of consecutive k, the run totals are scanned
// (wave shuffles, then the wave totals), and each thread walks its run
// again calling out(k, sum of val(0 .. k-1)); out(n, total) once.  val(k)
// is read before out(k) is called, by the same thread.
template <int BT, class Val, class Out>
__device__ __forceinline__ void block_scan(int n, int* wsum /* BT / 64 */, Val val, Out out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int per = (n + BT - 1) / BT;
    const int k0 = min((int)threadIdx.x * per, n), k1 = min(k0 + per, n);
    int run = 0;
    for (int k = k0; k < k1; ++k) run += val(k);
    int x = run;  // inclusive scan of the run totals within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int excl = x - run;
    for (int w = 0; w < wv; ++w) excl += wsum[w];
    int total = 0;
    for (int w = 0; w < BT / 64; ++w) total += wsum[w];
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
        const int v = val(k);
        out(k, excl);
        excl += v;
    }
    if (threadIdx.x == 0) out(n, total);
}

// Position r = h s of a fractional coordinate in the in-plane cell, with a
// fixed rounding sequence (the binning and the force kernel must agree to
// the bit: a particle finds itself at distance exactly zero).
template <typename real>
__device__ __forceinline__ void cell_position(real s0, real s1, real s2, real h00, real h01, real h10, real h11,
                                              real h22, real& x, real& y, real& z) {
    x = fma(h01, s1, h00 * s0);
    y = fma(h11, s1, h10 * s0);
    z = h22 * s2;
}

// From the cell counts cnt[0 .. ncell) of box b (LDS): the cell starts
// (cell_start and cnt[k] <- start of cell k, cnt[ncell] <- n), then the
// search layout's starts (gcell_start) and every column's offsets from cell
// order to its three segments of the search layout (col_off: the column's
// cells, lo_off: the image of its top zsub cells below it, hi_off: the image
// of its bottom zsub cells above it).  Ends with a barrier.
template <int BT>
__device__ void search_layout(const Ctx& C, const BoxInfo& B, const BoxDyn& D, int ncell, int* cnt, int* col_off,
                              int* lo_off, int* hi_off, int* wsum) {
    int* start = C.cell_start + B.cell_off;
    int* gstart = C.gcell_start + B.gcell_off;
    block_scan<BT>(ncell, wsum, [&](int k) { return cnt[k]; }, [&](int k, int excl) {
        start[k] = excl;
        cnt[k] = excl;
    });
    __syncthreads();
    const int n2 = D.nc[2], zs = B.zsub, gn2 = n2 + 2 * zs, ncol = D.nc[0] * D.nc[1];
    const float inv_gn2 = 1.0f / (float)gn2;
    // images before each column (its top and bottom zsub cells' particles
    // appear once more), scanned over columns
    __shared__ int n_images;
    block_scan<BT>(
        ncol, wsum,
        [&](int col) {
            const int k = col * n2;
            return (cnt[k + n2] - cnt[k + n2 - zs]) + (cnt[k + zs] - cnt[k]);
        },
        [&](int col, int excl) {
            if (col == ncol) {
                n_images = excl;
                return;
            }
            const int k = col * n2;
            const int first = cnt[k] + excl, top = cnt[k + n2] - cnt[k + n2 - zs];
            lo_off[col] = first - cnt[k + n2 - zs];
            col_off[col] = first + top - cnt[k];
            hi_off[col] = first + top + (cnt[k + n2] - cnt[k]) - cnt[k];
        });
    __syncthreads();
    // starts of the search-layout cells: a segment's offset plus the start
    // of the cell it repeats
    for (int g = threadIdx.x; g < ncol * gn2; g += BT) {
        const int col = div_small(g, inv_gn2), zg = g - col * gn2, k = col * n2;
        gstart[g] = zg < zs ? lo_off[col] + cnt[k + n2 - zs + zg]
                            : (zg < zs + n2 ? col_off[col] + cnt[k + zg - zs] : hi_off[col] + cnt[k + zg - zs - n2]);
    }
    if (threadIdx.x == 0) gstart[ncol * gn2] = B.n + n_images;
    __threadfence_block();
    __syncthreads();
}

// One workgroup per box: counting sort by cell in LDS, writing each
// particle's velocity record (velocity, local index) in cell order, sorted by
// index inside every cell so all later sums have a fixed order, and its
// position record (position, cell-order position) in the search layout: the
// same order per cell, plus the z images of bottom and top cells.
// LDS (dynamic): lds_cells cell counters / starts, three arrays of
// lds_cols column offsets (from cell order to the search layout:
// the column's cells, the image of its top cell, the image of its bottom
// cell), then room for lds_parts ints.  A box with at most lds_parts
// particles is scattered as entries into LDS, each thread ranks its own
// particles inside their cells and stores their records; a larger box
// scatters records to global scratch and sorts them there.  Both give the
// same records in the same order.
//
// fuse >= 0: the workgroup first runs the box's cell step and the half kick
// and drift of its particles (advance = fuse), counting cells as it goes;
// fuse < 0: k_cell_step and k_kick_drift have run.
template <typename real, int BIN_THREADS>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_box(Ctx C, int lds_cells, int lds_cols, int lds_parts, int fuse) {
    using R = Rec<real>;
    extern __shared__ int lds[];
    int* cnt = lds;
    int* col_off = lds + lds_cells;
    int* lo_off = col_off + lds_cols;
    int* hi_off = lo_off + lds_cols;
    int* lidx = hi_off + lds_cols;
    __shared__ int wsum[BIN_THREADS / 64];
    const int b = C.sel ? C.sel[blockIdx.x] : (int)blockIdx.x;
    const BoxInfo B = C.box[b];
    if (fuse >= 0) {
        if (threadIdx.x == 0) cell_step_box(C, b, fuse);
        __threadfence_block();
        __syncthreads();
    }
    const BoxDyn& D = C.dyn[b];
    const int ncell = D.nc[0] * D.nc[1] * D.nc[2];
    for (int k = threadIdx.x; k < ncell; k += BIN_THREADS) cnt[k] = 0;
    __syncthreads();
    const int* pc = C.pcell + B.off;
    // cells of this thread's particles k = threadIdx.x + j BIN_THREADS, kept
    // for the scatter when the box fits the LDS path
    constexpr int KEEP = 16384 / BIN_THREADS;
    int mycell[KEEP];
    const bool keep = B.n <= lds_parts && B.n <= KEEP * BIN_THREADS;
    if (fuse >= 0) {
        const KickDrift<real> K(C, D, B.rng_id);
        real* s = (real*)C.s;
        real* c = (real*)C.c;
        const real* f = (const real*)C.f;
        const int N = C.n_total;
        // four particles per thread and pass: all their loads issued before
        // any store, so the loads stay in flight together
#pragma unroll
        for (int j0 = 0; j0 < KEEP; j0 += 4) {
            if ((int)threadIdx.x + j0 * BIN_THREADS >= B.n) break;
            int cell[4];
            real sv[4][3], cv[4][3], fv[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = (int)threadIdx.x + (j0 + u) * BIN_THREADS;
                const int i = B.off + (k < B.n ? k : 0);
                for (int a = 0; a < 3; ++a) {
                    sv[u][a] = s[a * N + i];
                    cv[u][a] = c[a * N + i];
                    fv[u][a] = f[a * N + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = (int)threadIdx.x + (j0 + u) * BIN_THREADS;
                const int i = B.off + k;
                cell[u] = -1;
                if (k < B.n) {
                    if (fuse) {
                        kick_drift<real>(K, sv[u], cv[u], fv[u], k);
                        for (int a = 0; a < 3; ++a) {
                            c[a * N + i] = cv[u][a];
                            s[a * N + i] = sv[u][a];
                        }
                    }
                    cell[u] = cell_of(sv[u][0], sv[u][1], sv[u][2], K.nc);
                    if (!keep) C.pcell[i] = cell[u];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mycell[j0 + u] = cell[u];
                if (cell[u] >= 0) atomicAdd(&cnt[cell[u]], 1);
            }
        }
        for (int k = (int)threadIdx.x + KEEP * BIN_THREADS; k < B.n; k += BIN_THREADS)
            atomicAdd(&cnt[kick_drift_particle<real>(C, K, B.off + k, k, fuse)], 1);
        __threadfence_block();
    } else {
#pragma unroll
        for (int j0 = 0; j0 < KEEP; j0 += 4) {
            if ((int)threadIdx.x + j0 * BIN_THREADS >= B.n) break;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = (int)threadIdx.x + (j0 + u) * BIN_THREADS;
                mycell[j0 + u] = k < B.n ? pc[k] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (mycell[j0 + u] >= 0) atomicAdd(&cnt[mycell[j0 + u]], 1);
        }
        for (int k = (int)threadIdx.x + KEEP * BIN_THREADS; k < B.n; k += BIN_THREADS) atomicAdd(&cnt[pc[k]], 1);
    }
    __syncthreads();
    search_layout<BIN_THREADS>(C, B, D, ncell, cnt, col_off, lo_off, hi_off, wsum);
    const int* start = C.cell_start + B.cell_off;
    const int n2 = D.nc[2], zs = B.zsub;
    typename R::T* pv = (typename R::T*)C.cell_pv + 2 * (size_t)B.off;
    typename R::T* srec = (typename R::T*)C.srec + 2 * B.off;
    const real* s = (const real*)C.s;
    const real* c = (const real*)C.c;
    const int N = C.n_total;
    const real h00 = (real)D.h[0], h01 = (real)D.h[1], h10 = (real)D.h[3], h11 = (real)D.h[4];
    const real h22 = (real)D.h[8];
    // the position record of cell-order position q (cell `cell`) in its
    // search-layout slot and, for the zsub bottom or top cells, its image's slot
    const float inv_n2 = 1.0f / (float)n2;
    auto write_search = [&](int q, int cell, real x, real y, real z) {
        const int col = div_small(cell, inv_n2), zc = cell - col * n2;
        srec[q + col_off[col]] = R::make(x, y, z, q << 5);
        if (zc >= n2 - zs) srec[q + lo_off[col]] = R::make(x, y, z - h22, (q << 5) | 9);
        if (zc < zs) srec[q + hi_off[col]] = R::make(x, y, z + h22, (q << 5) | 18);
    };
    if (keep) {
        // LDS entries: cell << 14 | local index (cells < 2^14, particles < 2^14)
        int slot[KEEP];
#pragma unroll
        for (int j = 0; j < KEEP; ++j) {
            const int k = (int)threadIdx.x + j * BIN_THREADS;
            slot[j] = k < B.n ? atomicAdd(&cnt[mycell[j]], 1) : -1;
        }
#pragma unroll
        for (int j = 0; j < KEEP; ++j)
            if (slot[j] >= 0) lidx[slot[j]] = (mycell[j] << 14) | ((int)threadIdx.x + j * BIN_THREADS);
        __syncthreads();
        // cnt[k] now ends cell k: a particle's cell-order position is its
        // cell's start plus the number of its cell's entries with a smaller
        // index (a few each), so every cell is in index order
#pragma unroll
        for (int j = 0; j < KEEP; ++j) {
            if (slot[j] < 0) continue;
            const int cell = mycell[j], key = (cell << 14) | ((int)threadIdx.x + j * BIN_THREADS);
            const int q0 = cell == 0 ? 0 : cnt[cell - 1], q1 = cnt[cell];
            int rank = 0;
            for (int q = q0; q < q1; ++q) rank += lidx[q] < key;
            slot[j] = q0 + rank;
        }
        // the thread's own particles, four per pass with their (coalesced)
        // loads in flight together, each record stored to its slot
#pragma unroll
        for (int j0 = 0; j0 < KEEP; j0 += 4) {
            if ((int)threadIdx.x + j0 * BIN_THREADS >= B.n) break;
            real v[4][6];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = (int)threadIdx.x + (j0 + u) * BIN_THREADS;
                const int g = B.off + (k < B.n ? k : 0);
                v[u][0] = s[g]; v[u][1] = s[N + g]; v[u][2] = s[2 * N + g];
                v[u][3] = c[g]; v[u][4] = c[N + g]; v[u][5] = c[2 * N + g];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = (int)threadIdx.x + (j0 + u) * BIN_THREADS;
                if (k < B.n) {
                    const int q = slot[j0 + u];
                    real x, y, z;
                    cell_position<real>(v[u][0], v[u][1], v[u][2], h00, h01, h10, h11, h22, x, y, z);
                    pv[2 * q] = R::make(x, y, z, k);
                    pv[2 * q + 1] = R::make(v[u][3], v[u][4], v[u][5], k);
                    write_search(q, mycell[j0 + u], x, y, z);
                }
            }
        }
        return;
    }
    for (int k = threadIdx.x; k < B.n; k += BIN_THREADS) {
        const int pos = atomicAdd(&cnt[pc[k]], 1);
        const int g = B.off + k;
        real x, y, z;
        cell_position<real>(s[g], s[N + g], s[2 * N + g], h00, h01, h10, h11, h22, x, y, z);
        pv[2 * pos] = R::make(x, y, z, k);
    }
    __threadfence_block();
    __syncthreads();
    for (int k = threadIdx.x; k < ncell; k += BIN_THREADS) {
        const int q0 = start[k], q1 = start[k + 1];
        for (int q = q0 + 1; q < q1; ++q) {  // insertion sort by index, a few entries
            const typename R::T v = pv[2 * q];
            const int key = R::id(v);
            int r = q - 1;
            while (r >= q0 && R::id(pv[2 * r]) > key) {
                pv[2 * (r + 1)] = pv[2 * r];
                --r;
            }
            pv[2 * (r + 1)] = v;
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int q = threadIdx.x; q < B.n; q += BIN_THREADS) {
        const typename R::T v = pv[2 * q];
        const int k = R::id(v), g = B.off + k;
        pv[2 * q + 1] = R::make(c[g], c[N + g], c[2 * N + g], k);
        write_search(q, pc[k], v.x, v.y, v.z);
    }
}

// Binning of large boxes over several workgroups each.  The selected boxes
// (C.sel) are cut into chunks of `chunk` consecutive particles; per step:
//   k_cell_step (one thread per box), then
//   k_bin_count   (one workgroup per chunk): half kick and drift of the
//                 chunk's particles, their cells (pcell), the chunk's cell
//                 counts (cnt, one row of `cap` ints per chunk);
//   k_bin_scan    (one workgroup per box): the box's cell starts and search
//                 layout from the summed counts, each chunk's first position
//                 in every cell (off: the cell's start plus the counts of the
//                 box's earlier chunks) and the column offsets (col);
//   k_bin_scatter (one workgroup per chunk): each particle's position is its
//                 chunk's offset in its cell plus the number of the chunk's
//                 particles in that cell with a smaller index, so every cell
//                 is in index order as in k_bin_box, and the records are
//                 stored as k_bin_box stores them.
// The results equal k_bin_box's bit for bit.
struct SplitArgs {
    const int* box_chunk0;  // n_sel + 1: first chunk of each selected box
    const int* chunk_boxj;  // n_chunks: the selected box (index into C.sel) of each chunk
    int* cnt;               // n_chunks x cap: the chunk's particles per cell
    int* off;               // n_chunks x cap: the chunk's first position in each cell
    int* col;               // n_sel x 3 colcap: col_off, lo_off, hi_off per column
    int chunk, cap, colcap;
};

constexpr int SPLIT_BT = 1024;  // threads per workgroup of the split binning
constexpr int SPLIT_PER = 4;    // particles per thread and chunk at most (chunk <= 4096)

template <typename real>
__global__ __launch_bounds__(SPLIT_BT) void k_bin_count(Ctx C, SplitArgs S) {
    extern __shared__ int lds[];
    int* cnt = lds;
    const int k = blockIdx.x, j = S.chunk_boxj[k], b = C.sel[j];
    const BoxInfo B = C.box[b];
    const BoxDyn& D = C.dyn[b];
    const int first = (k - S.box_chunk0[j]) * S.chunk, last = min(first + S.chunk, B.n);
    const int ncell = D.nc[0] * D.nc[1] * D.nc[2];
    for (int q = threadIdx.x; q < ncell; q += SPLIT_BT) cnt[q] = 0;
    __syncthreads();
    const KickDrift<real> K(C, D, B.rng_id);
    for (int q = first + (int)threadIdx.x; q < last; q += SPLIT_BT)
        atomicAdd(&cnt[kick_drift_particle<real>(C, K, B.off + q, q, 1)], 1);
    __syncthreads();
    int* out = S.cnt + (size_t)k * S.cap;
    for (int q = threadIdx.x; q < ncell; q += SPLIT_BT) out[q] = cnt[q];
}

__global__ __launch_bounds__(SPLIT_BT) void k_bin_scan(Ctx C, SplitArgs S, int lds_cells, int lds_cols) {
    extern __shared__ int lds[];
    int* cnt = lds;
    int* col_off = lds + lds_cells;
    int* lo_off = col_off + lds_cols;
    int* hi_off = lo_off + lds_cols;
    __shared__ int wsum[SPLIT_BT / 64];
    const int j = blockIdx.x, b = C.sel[j];
    const BoxInfo B = C.box[b];
    const BoxDyn& D = C.dyn[b];
    const int ncell = D.nc[0] * D.nc[1] * D.nc[2];
    const int k0 = S.box_chunk0[j], k1 = S.box_chunk0[j + 1];
    for (int q = threadIdx.x; q < ncell; q += SPLIT_BT) {
        int t = 0;
        for (int k = k0; k < k1; ++k) t += S.cnt[(size_t)k * S.cap + q];
        cnt[q] = t;
    }
    __syncthreads();
    search_layout<SPLIT_BT>(C, B, D, ncell, cnt, col_off, lo_off, hi_off, wsum);
    for (int q = threadIdx.x; q < ncell; q += SPLIT_BT) {
        int run = cnt[q];
        for (int k = k0; k < k1; ++k) {
            S.off[(size_t)k * S.cap + q] = run;
            run += S.cnt[(size_t)k * S.cap + q];
        }
    }
    const int ncol = D.nc[0] * D.nc[1];
    int* col = S.col + (size_t)j * 3 * S.colcap;
    for (int q = threadIdx.x; q < ncol; q += SPLIT_BT) {
        col[q] = col_off[q];
        col[S.colcap + q] = lo_off[q];
        col[2 * S.colcap + q] = hi_off[q];
    }
}

template <typename real>
__global__ __launch_bounds__(SPLIT_BT) void k_bin_scatter(Ctx C, SplitArgs S) {
    using R = Rec<real>;
    extern __shared__ int lds[];
    int* lst = lds;          // cap: the chunk's local cell starts, then ends
    int* ent = lds + S.cap;  // chunk: local indices in local cell order
    __shared__ int wsum[SPLIT_BT / 64];
    const int k = blockIdx.x, j = S.chunk_boxj[k], b = C.sel[j];
    const BoxInfo B = C.box[b];
    const BoxDyn& D = C.dyn[b];
    const int first = (k - S.box_chunk0[j]) * S.chunk, last = min(first + S.chunk, B.n);
    const int ncell = D.nc[0] * D.nc[1] * D.nc[2];
    const int* ccnt = S.cnt + (size_t)k * S.cap;
    const int* coff = S.off + (size_t)k * S.cap;
    block_scan<SPLIT_BT>(ncell, wsum, [&](int q) { return ccnt[q]; }, [&](int q, int excl) {
        if (q < ncell) lst[q] = excl;
    });
    __syncthreads();
    const int* pc = C.pcell + B.off;
    int mycell[SPLIT_PER], slot[SPLIT_PER];
#pragma unroll
    for (int u = 0; u < SPLIT_PER; ++u) {
        const int q = first + (int)threadIdx.x + u * SPLIT_BT;
        mycell[u] = q < last ? pc[q] : -1;
        slot[u] = q < last ? atomicAdd(&lst[mycell[u]], 1) : -1;
    }
#pragma unroll
    for (int u = 0; u < SPLIT_PER; ++u)
        if (slot[u] >= 0) ent[slot[u]] = first + (int)threadIdx.x + u * SPLIT_BT;
    __syncthreads();
    // lst[c] now ends the chunk's entries of cell c
#pragma unroll
    for (int u = 0; u < SPLIT_PER; ++u) {
        if (slot[u] < 0) continue;
        const int c = mycell[u], me = first + (int)threadIdx.x + u * SPLIT_BT;
        const int e1 = lst[c], e0 = e1 - ccnt[c];
        int rank = 0;
        for (int e = e0; e < e1; ++e) rank += ent[e] < me;
        slot[u] = coff[c] + rank;
    }
    typename R::T* pv = (typename R::T*)C.cell_pv + 2 * (size_t)B.off;
    typename R::T* srec = (typename R::T*)C.srec + 2 * B.off;
    const real* s = (const real*)C.s;
    const real* cv = (const real*)C.c;
    const int N = C.n_total;
    const real h00 = (real)D.h[0], h01 = (real)D.h[1], h10 = (real)D.h[3], h11 = (real)D.h[4];
    const real h22 = (real)D.h[8];
    const int n2 = D.nc[2], zs = B.zsub;
    const float inv_n2 = 1.0f / (float)n2;
    const int* col = S.col + (size_t)j * 3 * S.colcap;
    real v[SPLIT_PER][6];
#pragma unroll
    for (int u = 0; u < SPLIT_PER; ++u) {
        const int q = first + (int)threadIdx.x + u * SPLIT_BT;
        const int g = B.off + (q < last ? q : first);
        v[u][0] = s[g]; v[u][1] = s[N + g]; v[u][2] = s[2 * N + g];
        v[u][3] = cv[g]; v[u][4] = cv[N + g]; v[u][5] = cv[2 * N + g];
    }
#pragma unroll
    for (int u = 0; u < SPLIT_PER; ++u) {
        if (slot[u] < 0) continue;
        const int q = first + (int)threadIdx.x + u * SPLIT_BT, pos = slot[u];
        real x, y, z;
        cell_position<real>(v[u][0], v[u][1], v[u][2], h00, h01, h10, h11, h22, x, y, z);
        pv[2 * pos] = R::make(x, y, z, q);
        pv[2 * pos + 1] = R::make(v[u][3], v[u][4], v[u][5], q);
        const int cc = div_small(mycell[u], inv_n2), zc = mycell[u] - cc * n2;
        srec[pos + col[cc]] = R::make(x, y, z, pos << 5);
        if (zc >= n2 - zs) srec[pos + col[S.colcap + cc]] = R::make(x, y, z - h22, (pos << 5) | 9);
        if (zc < zs) srec[pos + col[2 * S.colcap + cc]] = R::make(x, y, z + h22, (pos << 5) | 18);
    }
}

// In-plane image shift sh0 a + sh1 b of the cell's lattice vectors for the
// code ic = 3 (sh0 + 1) + (sh1 + 1) (0 .. 8), with a fixed rounding sequence:
// the search and the evaluation of a pair form the same separation.
template <typename real>
__device__ __forceinline__ void image_shift(int ic, real h00, real h01, real h10, real h11, real& sx, real& sy) {
    const int c0 = (ic * 11) >> 5;  // ic / 3 for 0 <= ic <= 8
    const real a = (real)(c0 - 1), b = (real)(ic - 3 * c0 - 1);
    sx = fma(h01, b, h00 * a);
    sy = fma(h11, b, h10 * a);
}

template <typename real>
__device__ __forceinline__ real inv_sqrt(real x);
template <>
__device__ __forceinline__ float inv_sqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double inv_sqrt<double>(double x) { return 1.0 / sqrt(x); }

// Pair forces (Eqs. conservative, dissipative, random) and FENE bonds (Eq.
// fene_force).  Each lane owns one particle in cell order and sums that
// particle's force in registers, so every ordered pair is evaluated by its
// first particle's lane: no atomics, and a fixed summation order.
//   Search: the wave walks the nine stencil rows in step (z cells
//   k2 - zsub .. k2 + zsub of a row, periodic images included, are one
//   contiguous range of the search layout; with two cells per cutoff along z
//   the rows hold ~20% fewer candidates); each lane scans its own row range
//   SU records at a time (lanes of one home cell read the same records) and
//   appends each accepted neighbour (0 < r < rc; the particle itself has
//   r = 0) to its own LDS queue of QD four-byte entries: the neighbour's
//   cell-order position and its image code.  QD, `drain` and `busy` are
//   tuning parameters; none changes the order in which a lane evaluates its
//   neighbours, so results do not depend on them.
//   Evaluation: a round pops one queued neighbour per lane, reloads its
//   position and velocity records, re-forms the separation with the same
//   rounding as the search, and evaluates the pair (relative velocity
//   including the streaming difference L d, Philox normal, force, virial).
//   Rounds run when a queue could overflow, until every queue holds at most
//   `drain` entries (and while `busy` or more lanes have work), and the
//   queues are drained at the end.  Deep queues let most lanes hold work in
//   every round; the float kernel is bounded to 96 VGPRs so five waves share
//   each SIMD (the loop is latency-bound).
// records tested per lane and search iteration for a queue of depth QD
__host__ __device__ constexpr int scan_unroll(int qd) { return qd >= 8 ? 4 : (qd >= 4 ? 2 : 1); }

// Fraction of the in-plane segment a + t e, t in [0, 1], inside the square
// |x|, |y| <= hc (the bond function of a weight uniform over a
// boundary-region box's core, times the core's volume).
template <typename real>
__device__ __forceinline__ real core_fraction(real ax, real ay, real ex, real ey, real hc) {
    real t0 = (real)0, t1 = (real)1;
    const real a[2] = {ax, ay}, e[2] = {ex, ey};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (e[k] == (real)0) {
            if (a[k] < -hc || a[k] > hc) return (real)0;
            continue;
        }
        real ta = (-hc - a[k]) / e[k], tb = (hc - a[k]) / e[k];
        if (ta > tb) {
            const real x = ta;
            ta = tb;
            tb = x;
        }
        t0 = fmax(t0, ta);
        t1 = fmin(t1, tb);
    }
    return t1 > t0 ? t1 - t0 : (real)0;
}

// PRUNE selects the stencil-pruning variant; without it the float kernel
// fits 80 VGPRs, six waves per SIMD.  COMP keeps the virials of the
// conservative, dissipative and random forces apart as well (their sum is
// accumulated as in the default variant), at the cost of 18 more registers.
// AF handles boxes with boundary regions: each pair's and bond's virial is
// weighted by the fraction of its segment inside the core, and the second
// half kick relaxes the ring toward the imposed field; the core's kinetic
// sums use the velocity relative to that field.
template <typename real, int QD, bool PRUNE, bool COMP = false, bool AF = false>
__global__ __launch_bounds__(BS, sizeof(real) == 4 ? (COMP || AF || QD >= 32 ? 4 : (PRUNE ? 5 : 6)) : 1) void k_forces(
    Ctx C, int step_offset, int drain, int busy, int kick) {
    constexpr bool prune = PRUNE;
    constexpr int NV = COMP ? 37 : 19;  // block partial sums
    using R = Rec<real>;
    using V4 = typename R::T;
    constexpr int NW = BS / 64;
    constexpr int SU = scan_unroll(QD);
    // queue entry: cell-order position of j << 5 | image code, the code
    // 9 x z image (0 none, 1 below, 2 above) + in-plane image code (0 .. 8)
    __shared__ int qbuf[QD][NW][64];
    __shared__ double red[NV * NW];
    // per image code (0 .. 26) the shift of the block's box: in-plane
    // image_shift, and 0, -h22 or +h22 along z
    __shared__ real shift_tab[32][4];

    int blk = xcd_local_work(blockIdx.x, gridDim.x);
    if (C.blk_list) blk = C.blk_list[blk];
    const int b = C.blk_box[blk];
    const BoxInfo B = C.box[b];
    const BoxDyn& D = C.dyn[b];
    const int N = C.n_total;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int p0 = C.blk_first[blk] - B.off;  // first cell-order position of the block
    const int pos = p0 + t;
    const bool act = pos < B.n;
    const V4* pv = (const V4*)C.cell_pv + 2 * (size_t)B.off;
    const char* sbase = (const char*)((const V4*)C.srec + 2 * B.off);
    const __amdgpu_buffer_rsrc_t srsrc = rec_rsrc(sbase);
    const real* s = (const real*)C.s;
    real* f = (real*)C.f;

    // in-plane cell and gradient
    const real h00 = (real)D.h[0], h01 = (real)D.h[1], h10 = (real)D.h[3], h11 = (real)D.h[4];
    const real h22 = (real)D.h[8];
    if (t < 27) {
        image_shift<real>(t % 9, h00, h01, h10, h11, shift_tab[t][0], shift_tab[t][1]);
        shift_tab[t][2] = t < 9 ? (real)0 : (t < 18 ? -h22 : h22);
    }
    __syncthreads();
    real ri0 = 0, ri1 = 0, ri2 = 0, ci0 = 0, ci1 = 0, ci2 = 0;
    real own_s0 = 0, own_s1 = 0, own_s2 = 0;
    int own_id = 0;
    if (act) {
        const V4 u = pv[2 * pos + 1];
        ci0 = u.x; ci1 = u.y; ci2 = u.z;
        own_id = R::id(u);
        const int g = B.off + own_id;
        own_s0 = s[g]; own_s1 = s[N + g]; own_s2 = s[2 * N + g];
        cell_position<real>(own_s0, own_s1, own_s2, h00, h01, h10, h11, h22, ri0, ri1, ri2);
    }
    const real L00 = (real)D.L[0], L01 = (real)D.L[1], L10 = (real)D.L[3], L11 = (real)D.L[4];
    // boundary regions: core half-width, the cell centre (r' = r - centre)
    const bool afbc = AF && D.hc > 0.0;
    const real hcr = AF ? (real)D.hc : (real)0;
    const real cx = AF ? (real)(0.5 * (D.h[0] + D.h[1])) : (real)0, cy = AF ? (real)(0.5 * (D.h[3] + D.h[4])) : (real)0;
    const int n0 = D.nc[0], n1 = D.nc[1], n2 = D.nc[2], zs = B.zsub;
    const real dzc = h22 / (real)n2;  // cell height
    auto sqr = [](real x) { return x * x; };
    const unsigned stepc = (unsigned)(*C.step + (unsigned long long)step_offset);
    const real a = (real)C.a, gam = (real)C.gamma, sig = (real)(C.sigma * C.rdt);
    const real rc2 = (real)C.rc2, irc = (real)(1.0 / C.rc);
    const int* gstart = C.gcell_start + B.gcell_off;

    int k0 = 0, k1 = 0, k2 = 0;
    if (act) cell_coords(own_s0, own_s1, own_s2, D.nc, k0, k1, k2);  // as the binning found it
    // Stencil pruning: distances from the particle to the planes bounding
    // its cell (fractional gap x perpendicular width of the cell); any point
    // of a neighbour cell across such a plane is at least that far away.  A
    // row (d0, d1) is skipped when its in-plane lower bound g reaches the
    // cutoff, and its cells below / above the particle's z cell are scanned
    // only if they may hold a point within sqrt(rc^2 - g^2).  Bounds are
    // compared with a 0.1% larger cutoff, so no pair within rc is dropped
    // and the scan order of the kept candidates is unchanged.
    real gl0 = 0, gh0 = 0, gl1 = 0, gh1 = 0, zl = 0, zh = 0;
    const real rcp2 = prune ? (real)(1.002 * C.rc2) : (real)0;
    if (act && prune) {
        const int gi = B.off + own_id;
        const real s0 = s[gi], s1 = s[N + gi], s2 = s[2 * N + gi];
        const real area = fabs(h00 * h11 - h01 * h10);
        const real w0 = area / sqrt(h01 * h01 + h11 * h11), w1 = area / sqrt(h00 * h00 + h10 * h10);
        const real f0 = s0 * (real)n0 - (real)k0, f1 = s1 * (real)n1 - (real)k1, f2 = s2 * (real)n2 - (real)k2;
        gl0 = fmax(f0, (real)0) * w0 / (real)n0;
        gh0 = fmax((real)1 - f0, (real)0) * w0 / (real)n0;
        gl1 = fmax(f1, (real)0) * w1 / (real)n1;
        gh1 = fmax((real)1 - f1, (real)0) * w1 / (real)n1;
        zl = fmax(f2, (real)0) * h22 / (real)n2;
        zh = fmax((real)1 - f2, (real)0) * h22 / (real)n2;
    }
    // this lane's queue: entries popped and pushed, counted in queue rows
    // (NW x 64 ints) so that an entry's LDS byte address is one and-or of the
    // count with the lane's offset
    constexpr unsigned QROW = NW * 64 * sizeof(int), QMASK = (QD - 1) * QROW;
    const unsigned qlane = (unsigned)t * sizeof(int);
    char* const qbase = (char*)&qbuf[0][0][0];
    unsigned qh = 0, qt = 0;
    real fx = 0, fy = 0, fz = 0;
    real w[6] = {0, 0, 0, 0, 0, 0};
    real wc[COMP ? 6 : 1] = {}, wd[COMP ? 6 : 1] = {}, wr[COMP ? 6 : 1] = {};  // C, D, R parts

    int ic = 4;  // in-plane image code of the row being scanned
    // one evaluation round: each lane with a queued neighbour takes the oldest
    auto round = [&]() {
        if (qt > qh) {
            const int e = *(const int*)(qbase + ((qh & QMASK) | qlane));
            qh += QROW;
            // one 32-bit byte offset from the box's records (scalar base)
            const unsigned po = ((unsigned)e >> 5) * (unsigned)(2 * sizeof(V4));
            const V4 pj = *(const V4*)((const char*)pv + po);
            const V4 cj = *(const V4*)((const char*)pv + po + sizeof(V4));
            const int code = e & 31;
            const real sx = shift_tab[code][0], sy = shift_tab[code][1];
            // the z image: one rounding of z + (0, -h22, +h22), the same as the
            // binning's z - h22, z + h22
            const real zj = pj.z + shift_tab[code][2];
            const real dx = (ri0 - sx) - pj.x, dy = (ri1 - sy) - pj.y, dz = ri2 - zj;
            const real r2 = fma(dz, dz, fma(dx, dx, dy * dy));  // fixed association
            const real ir = inv_sqrt(r2);
            const real r = r2 * ir;
            const real ex = dx * ir, ey = dy * ir, ez = dz * ir;
            const real wR = (real)1 - r * irc;
            const real vx = ci0 - cj.x + L00 * dx + L01 * dy;
            const real vy = ci1 - cj.y + L10 * dx + L11 * dy;
            const real vz = ci2 - cj.z;
            const real ev = ex * vx + ey * vy + ez * vz;
            const real th = pair_theta<real>((unsigned)own_id, (unsigned)R::id(cj), stepc, B.rng_id, C.key0, C.key1);
            const real mag = wR * (a - gam * wR * ev + sig * th);
            const real gx = mag * ex, gy = mag * ey, gz = mag * ez;
            fx += gx; fy += gy; fz += gz;
            // a boundary-region box weighs the pair by its segment's share of the core
            const real wgt = afbc ? core_fraction<real>(ri0 - cx, ri1 - cy, -dx, -dy, hcr) : (real)1;
            const real dxw = AF ? dx * wgt : dx, dyw = AF ? dy * wgt : dy, dzw = AF ? dz * wgt : dz;
            w[0] += dxw * gx; w[1] += dyw * gy; w[2] += dzw * gz;
            w[3] += dxw * gy; w[4] += dxw * gz; w[5] += dyw * gz;
            if constexpr (COMP) {
                // d (x) e times each force's magnitude
                const real mc = wR * a, md = -(wR * gam * wR * ev), mr = wR * sig * th;
                const real de[6] = {dxw * ex, dyw * ey, dzw * ez, dxw * ey, dxw * ez, dyw * ez};
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    wc[k] += mc * de[k];
                    wd[k] += md * de[k];
                    wr[k] += mr * de[k];
                }
            }
        }
    };
    // test one candidate record v against (px, py, pz), the lane's
    // position minus the image shift of the range scanned; queue it if accepted
    auto push = [&](bool valid, const V4& v, real px, real py, real pz) {
        const real dx = px - v.x, dy = py - v.y, dz = pz - v.z;
        // the acceptance test's rounding is fixed by explicit fmas, whatever the
        // surrounding code lets the compiler contract
        const real r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        // one branch per candidate: the tests combined without short-circuit
        if (valid & (r2 < rc2) & (r2 > (real)0)) {
            *(int*)(qbase + ((qt & QMASK) | qlane)) = R::id(v) + ic;
            qt += QROW;
        }
    };

    // Scan state: the wave is at stencil row `row` (d0, d1); each lane scans
    // the search-layout records q .. qe-1 (z cells k2 - zsub .. k2 + zsub of
    // the row's column, the periodic images included) against (bx, by, ri2), its
    // position less the in-plane image shift of the column.
    int row = 0;
    int q = 0, qe = 0;
    real bx = 0, by = 0;
    auto set_range = [&]() {
        const int d0 = row / 3 - 1, d1 = row % 3 - 1;
        int m0 = k0 + d0, m1 = k1 + d1;
        const int sh0 = m0 < 0 ? -1 : (m0 >= n0 ? 1 : 0);
        const int sh1 = m1 < 0 ? -1 : (m1 >= n1 ? 1 : 0);
        m0 -= sh0 * n0;
        m1 -= sh1 * n1;
        const int gb = (m0 * n1 + m1) * (n2 + 2 * zs) + k2;
        ic = 3 * (sh0 + 1) + (sh1 + 1);
        bx = ri0 - shift_tab[ic][0];
        by = ri1 - shift_tab[ic][1];
        q = 0;
        qe = 0;
        int lo = 0, hi = 2 * zs + 1;
        bool live = act;
        if (act && prune) {
            const real ga = d0 < 0 ? gl0 : (d0 > 0 ? gh0 : (real)0);
            const real gb2 = d1 < 0 ? gl1 : (d1 > 0 ? gh1 : (real)0);
            const real g = fmax(ga, gb2);
            const real zmax2 = rcp2 - g * g;
            live = zmax2 > (real)0;
            // z cells below (above) the particle's, farthest first
            for (int j = zs; j >= 1 && !(sqr(zl + (real)(j - 1) * dzc) < zmax2); --j) ++lo;
            for (int j = zs; j >= 1 && !(sqr(zh + (real)(j - 1) * dzc) < zmax2); --j) --hi;
        }
        if (live) {
            q = gstart[gb + lo];
            qe = gstart[gb + hi];
        }
    };
    set_range();
    bool scanning = true;  // wave-uniform
    while (true) {
        // search until the stencil is done or some queue might not take two more
        while (scanning) {
            if (__ballot(q < qe) == 0ull) {
                if (++row == 9) {
                    scanning = false;
                    break;
                }
                set_range();
                continue;
            }
            // SU records per lane per iteration, all loads issued before the
            // first test, addressed by one 32-bit byte offset from the box's
            // records; slots past the range end read the next records (the
            // array is padded) and are discarded
            V4 cand[SU];
            const unsigned qo = (unsigned)q * (unsigned)sizeof(V4);
            const int rem = qe - q;
#pragma unroll
            for (int u = 0; u < SU; ++u) cand[u] = load_rec<real>(srsrc, sbase, qo + u * (unsigned)sizeof(V4));
#pragma unroll
            for (int u = 0; u < SU; ++u) push(u < rem, cand[u], bx, by, ri2);
            q += SU;
            // evaluate when a queue may not take SU more, or when enough
            // lanes hold a neighbour for a well-filled round
            if (__ballot(qt - qh > (QD - SU) * QROW) != 0ull || __popcll(__ballot(qt > qh)) >= busy) break;
        }
        if (!scanning) {
            while (__ballot(qt > qh) != 0ull) round();
            break;
        }
        // evaluate until every queue holds at most `drain` entries and fewer
        // than `busy` lanes hold one
        do {
            round();
        } while (__ballot(qt - qh > (unsigned)drain * QROW) != 0ull || __popcll(__ballot(qt > qh)) >= busy);
    }

    real wf[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        const int i = B.off + own_id;
        // FENE springs to the chain neighbours
        if (own_id < B.n_beads) {
            const real si0 = s[i], si1 = s[N + i], si2 = s[2 * N + i];
            const int bead = own_id % C.chain_len;
            const real Hf = (real)C.H, iR02 = (real)C.inv_R02;
            for (int side = 0; side < 2; ++side) {
                if (side == 0 && bead == 0) continue;
                if (side == 1 && bead == C.chain_len - 1) continue;
                const int j = side == 0 ? i - 1 : i + 1;
                real ds0 = si0 - s[j], ds1 = si1 - s[N + j], ds2 = si2 - s[2 * N + j];
                ds0 -= rint(ds0); ds1 -= rint(ds1); ds2 -= rint(ds2);
                const real dx = h00 * ds0 + h01 * ds1, dy = h10 * ds0 + h11 * ds1, dz = h22 * ds2;
                real den = (real)1 - (dx * dx + dy * dy + dz * dz) * iR02;
                if (den <= (real)0) atomicOr(&C.flags[b], LHMM_FLAG_BOND);
                if (den < (real)0.01) den = (real)0.01;
                const real k = -Hf / den;
                const real gx = k * dx, gy = k * dy, gz = k * dz;
                fx += gx; fy += gy; fz += gz;
                if (side == 1) {  // each bond's virial once, by its lower bead
                    const real wgt = afbc ? core_fraction<real>(ri0 - cx, ri1 - cy, -dx, -dy, hcr) : (real)1;
                    const real dxw = AF ? dx * wgt : dx, dyw = AF ? dy * wgt : dy, dzw = AF ? dz * wgt : dz;
                    wf[0] += dxw * gx; wf[1] += dyw * gy; wf[2] += dzw * gz;
                    wf[3] += dxw * gy; wf[4] += dxw * gz; wf[5] += dyw * gz;
                }
            }
        }
        f[i] = fx; f[N + i] = fy; f[2 * N + i] = fz;
    }
    double v[NV];
    for (int k = 0; k < 6; ++k) {
        v[k] = (double)w[k];
        v[6 + k] = (double)wf[k];
        v[13 + k] = 0.0;
        if constexpr (COMP) {
            v[19 + k] = (double)wc[k];
            v[25 + k] = (double)wd[k];
            v[31 + k] = (double)wr[k];
        }
    }
    v[12] = (double)(qt / QROW);  // every queued neighbour was evaluated once
    // second half kick of the velocity-Verlet step, c += dt/2 (F/m - L c),
    // with the particle's final force, and the kinetic partial sums m c c
    if (kick && act) {
        const int i = B.off + own_id;
        real* c = (real*)C.c;
        const real hdt = (real)(0.5 * C.dt), im = (real)C.inv_mass;
        real c0 = ci0, c1 = ci1, c2 = ci2;
        const real lc0 = L00 * c0 + L01 * c1, lc1 = L10 * c0 + L11 * c1;
        c0 += hdt * (fx * im - lc0);
        c1 += hdt * (fy * im - lc1);
        c2 += hdt * (fz * im);
        bool in_core = true;
        real u0 = (real)0, u1 = (real)0;  // imposed field at the particle (boundary regions)
        if (afbc) {
            const real x = h00 * (own_s0 - (real)0.5) + h01 * (own_s1 - (real)0.5);
            const real y = h10 * (own_s0 - (real)0.5) + h11 * (own_s1 - (real)0.5);
            const real G[4] = {(real)D.G[0], (real)D.G[1], (real)D.G[2], (real)D.G[3]};
            ring_relax<real>(x, y, hcr, (real)D.hb, G, (real)C.ou_damp, (real)C.ou_amp, (unsigned)own_id, 1u, stepc,
                             B.rng_id, C.key0, C.key1, c0, c1);
            in_core = fmax(fabs(x), fabs(y)) < hcr;
            u0 = G[0] * x + G[1] * y;
            u1 = G[2] * x + G[3] * y;
        }
        c[i] = c0; c[N + i] = c1; c[2 * N + i] = c2;
        if (in_core) {
            const double mm = C.mass, x = (double)(c0 - u0), y = (double)(c1 - u1), z = (double)c2;
            v[13] = mm * x * x; v[14] = mm * y * y; v[15] = mm * z * z;
            v[16] = mm * x * y; v[17] = mm * x * z; v[18] = mm * y * z;
        }
    }
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 12; ++k) C.part_vir[(size_t)C.pv_stride * blk + k] = v[k];
        if constexpr (COMP)
            for (int k = 0; k < 18; ++k) C.part_vir[(size_t)C.pv_stride * blk + 12 + k] = v[19 + k];
        C.part_pairs[blk] = (unsigned)v[12];
        if (kick)
            for (int k = 0; k < 6; ++k) C.part_kin[6 * blk + k] = v[13 + k];
    }
}

// One wave per box: the step's stress, sigma = -(K + W)/V, by part.  Lane l
// sums the partials of blocks l, l+64, ...; a fixed shuffle tree combines
// the lanes, so the order of every sum is fixed.  With the C, D, R parts
// kept (pv_stride 30) they are reduced alongside.
__global__ __launch_bounds__(64) void k_box_stress(Ctx C) {
    const int b = C.sel ? C.sel[blockIdx.x] : (int)blockIdx.x;
    const int lane = threadIdx.x;
    const BoxInfo B = C.box[b];
    const bool comp = C.pv_stride > 12;
    double v[37];
    for (int q = 0; q < 37; ++q) v[q] = 0.0;
    for (int k = lane; k < B.nblk; k += 64) {
        const int blk = B.blk_off + k;
        for (int q = 0; q < 6; ++q) v[q] += C.part_kin[6 * blk + q];
        for (int q = 0; q < 12; ++q) v[6 + q] += C.part_vir[(size_t)C.pv_stride * blk + q];
        v[18] += (double)C.part_pairs[blk];
        if (comp)
            for (int q = 0; q < 18; ++q) v[19 + q] += C.part_vir[(size_t)C.pv_stride * blk + 12 + q];
    }
#pragma unroll
    for (int q = 0; q < 37; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if (lane == 0) {
        const double iv = 1.0 / C.dyn[b].vol;
        double* acc = C.acc + ACC * b;
        bool finite = true;
        for (int q = 0; q < 6; ++q) {
            const double sk = -v[q] * iv, sp = -C.vir_scale * v[6 + q] * iv, sf = -v[12 + q] * iv;
            acc[q] += sk;
            acc[6 + q] += sp;
            acc[12 + q] += sf;
            if (!(fabs(sk + sp + sf) <= 1e300)) finite = false;
            if (comp)
                for (int r = 0; r < 3; ++r) acc[18 + 6 * r + q] += -C.vir_scale * v[19 + 6 * r + q] * iv;
        }
        if (!finite) C.flags[b] |= LHMM_FLAG_NONFINITE;
        const unsigned long long np = (unsigned long long)v[18];
        const unsigned long long up = C.vir_scale < 1.0 ? np / 2 : np;
        C.acc_pairs[b] += up;
        C.tot_pairs[b] += up;
        if (blockIdx.x == 0) *C.step += 1ull;
    }
}

// Copy the snapshot state of the selected boxes back (one workgroup per box)
// and clear their flags.
template <typename real>
__global__ __launch_bounds__(256) void k_restore(Ctx C, const real* __restrict__ ss, const real* __restrict__ sc,
                                                 const real* __restrict__ sf, const BoxDyn* __restrict__ sdyn) {
    const int b = C.sel[blockIdx.x];
    const BoxInfo B = C.box[b];
    const int N = C.n_total;
    real* s = (real*)C.s;
    real* c = (real*)C.c;
    real* f = (real*)C.f;
    for (int k = 0; k < 3; ++k)
        for (int i = threadIdx.x; i < B.n; i += blockDim.x) {
            const long q = (long)k * N + B.off + i;
            s[q] = ss[q];
            c[q] = sc[q];
            f[q] = sf[q];
        }
    if (threadIdx.x == 0) {
        C.dyn[b] = sdyn[b];
        C.flags[b] = 0u;
    }
}

__global__ void k_finalize(Ctx C, double* __restrict__ stress_out, double* __restrict__ parts_out,
                           double inv_steps) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= C.n_boxes) return;
    const double* acc = C.acc + ACC * b;
    for (int q = 0; q < 6; ++q) stress_out[6 * b + q] = (acc[q] + acc[6 + q] + acc[12 + q]) * inv_steps;
    for (int q = 0; q < ACC; ++q) parts_out[ACC * b + q] = acc[q] * inv_steps;
}

}  // namespace

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------

struct lhmm_micro {
    lhmm_params p{};
    lhmm_micro_config cfg{};
    int bin_lds_cells = 0, bin_lds_cols = 0, bin_lds_parts = 0;  // dynamic LDS of the binning kernel (ints)
    int n_boxes = 0, n_blocks = 0, precision = LHMM_FP32;
    long long n_total = 0;
    size_t real_size = 4;
    std::vector<BoxInfo> box;
    std::vector<int> blk_box, blk_first;
    hipStream_t user_stream = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // device buffers
    BoxInfo* d_box = nullptr;
    BoxDyn* d_dyn = nullptr;
    unsigned* d_flags = nullptr;
    int *d_blk_box = nullptr, *d_blk_first = nullptr;
    void *d_s = nullptr, *d_c = nullptr, *d_f = nullptr;
    int *d_pcell = nullptr, *d_cell_start = nullptr, *d_gcell_start = nullptr;
    void* d_cell_pv = nullptr;
    void* d_srec = nullptr;
    double *d_part_vir = nullptr, *d_part_kin = nullptr;
    unsigned* d_part_pairs = nullptr;
    double *d_acc = nullptr, *d_parts = nullptr, *d_gradL = nullptr;
    unsigned long long *d_acc_pairs = nullptr, *d_tot_pairs = nullptr, *d_step = nullptr;
    unsigned long long* d_gstep = nullptr;  // step counters of the groups inside a captured chunk
    // selection lists (device) and their pinned staging, reused once ev_sel completes
    int *d_sel = nullptr, *d_blk_list = nullptr, *h_sel = nullptr;
    hipEvent_t ev_sel = nullptr;
    // snapshot of the particle state and per-box cells
    void *d_snap_s = nullptr, *d_snap_c = nullptr, *d_snap_f = nullptr;
    BoxDyn* d_snap_dyn = nullptr;
    bool have_snapshot = false;
    bool have_state = false, forces_valid = false;
    bool afbc = false;  // some box has boundary regions (lhmm_micro_set_afbc)
    std::map<int, hipGraphExec_t> graphs;
    // graphs of subset steps, keyed by (boxes, blocks, steps): a shape is
    // captured the second time it is asked for (history replays repeat it)
    std::map<std::tuple<int, int, int>, hipGraphExec_t> sub_graphs;
    std::map<std::tuple<int, int, int>, int> sub_seen;
    // overlapped groups of boxes (cfg.groups > 1): boxes by particle count,
    // smallest first; inside a captured chunk of steps each group runs all
    // its steps (binning, forces, stress) on its own stream with its own step
    // counter, and the groups join at the chunk's end
    struct Group {
        int* d_sel = nullptr;
        int* d_blk = nullptr;
        int n_sel = 0, nblk = 0, lds_cells = 0, lds_cols = 0, lds_parts = 0;
        // split binning (cfg.bin_split > 0, the group of the largest boxes)
        int n_chunks = 0;
        int* d_split = nullptr;  // box_chunk0, chunk_boxj, cnt, off, col in one allocation
        SplitArgs S{};
    };
    std::vector<Group> groups;
    hipStream_t aux[MAX_GROUPS - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[MAX_GROUPS - 1] = {};
    Ctx ctx{};
};

namespace {

// Column capacity of a box's cell grid: n0 n1 n2 <= cell_cap with
// n2 >= 2 zsub + 1, or n0, n1 <= 3 when the grid had to be clipped.
int box_cols(const BoxInfo& B) { return std::max(B.cell_cap / (2 * B.zsub + 1), 9) + 1; }

template <typename real>
void launch_bin(lhmm_micro* m, const Ctx& C, int nbox, hipStream_t st, int fuse, int lc = 0, int lcol = 0,
                int lp = 0) {
    if (lc == 0) {
        lc = m->bin_lds_cells;
        lcol = m->bin_lds_cols;
        lp = m->bin_lds_parts;
    }
    const size_t bytes = sizeof(int) * ((size_t)lc + 3 * (size_t)lcol + (size_t)lp);
    switch (m->cfg.bin_threads) {
        case 256: k_bin_box<real, 256><<<nbox, 256, bytes, st>>>(C, lc, lcol, lp, fuse); break;
        case 512: k_bin_box<real, 512><<<nbox, 512, bytes, st>>>(C, lc, lcol, lp, fuse); break;
        default: k_bin_box<real, 1024><<<nbox, 1024, bytes, st>>>(C, lc, lcol, lp, fuse); break;
    }
}

// kick = 1: a full step's force pass, which ends with the second half kick
template <typename real>
void launch_forces(lhmm_micro* m, const Ctx& C, int nblk, int step_offset, int kick, hipStream_t st) {
    const int drain = m->cfg.drain, busy = m->cfg.busy_lanes;
#define LHMM_FORCES(QD)                                                                              \
    do {                                                                                             \
        if (m->afbc && C.pv_stride > 12)                                                             \
            k_forces<real, QD, false, true, true><<<nblk, BS, 0, st>>>(C, step_offset, drain, busy, kick);  \
        else if (m->afbc)                                                                            \
            k_forces<real, QD, false, false, true><<<nblk, BS, 0, st>>>(C, step_offset, drain, busy, kick); \
        else if (C.pv_stride > 12)                                                                   \
            k_forces<real, QD, false, true><<<nblk, BS, 0, st>>>(C, step_offset, drain, busy, kick);        \
        else if (m->cfg.prune)                                                                       \
            k_forces<real, QD, true><<<nblk, BS, 0, st>>>(C, step_offset, drain, busy, kick);               \
        else                                                                                         \
            k_forces<real, QD, false><<<nblk, BS, 0, st>>>(C, step_offset, drain, busy, kick);              \
    } while (0)
    switch (m->cfg.queue_depth) {
        case 2: LHMM_FORCES(2); break;
        case 4: LHMM_FORCES(4); break;
        case 8: LHMM_FORCES(8); break;
        case 32: LHMM_FORCES(32); break;
        default: LHMM_FORCES(16); break;
    }
#undef LHMM_FORCES
}

// One step (or a force evaluation) of the boxes C selects: all n_boxes boxes
// and n_blocks work blocks, or the n_sel selected boxes and their nblk blocks.
template <typename real>
void launch_step_kernels(lhmm_micro* m, const Ctx& C, int nbox, int nblk, int step_offset, bool advance,
                         bool full_step) {
    const int bt = 256, bg = (nbox + bt - 1) / bt;
    if (m->cfg.fuse_bin) {
        launch_bin<real>(m, C, nbox, m->stream, advance ? 1 : 0);
    } else {
        k_cell_step<<<bg, bt, 0, m->stream>>>(C, advance ? 1 : 0);
        k_kick_drift<real><<<nblk, BS, 0, m->stream>>>(C, advance ? 1 : 0);
        launch_bin<real>(m, C, nbox, m->stream, -1);
    }
    launch_forces<real>(m, C, nblk, step_offset, full_step ? 1 : 0, m->stream);
    if (full_step) k_box_stress<<<nbox, 64, 0, m->stream>>>(C);
}

// One step with an event pair around each kernel (ev: 2 * LHMM_N_KERNELS events).
template <typename real>
void launch_step_timed(lhmm_micro* m, hipEvent_t* ev) {
    const Ctx& C = m->ctx;
    const int bt = 256, bg = (m->n_boxes + bt - 1) / bt;
    hipStream_t st = m->stream;
    // with the fused binning kernel the cell step and kick-drift pairs time nothing
    const bool fused = m->cfg.fuse_bin != 0;
    (void)hipEventRecord(ev[0], st);
    if (!fused) k_cell_step<<<bg, bt, 0, st>>>(C, 1);
    (void)hipEventRecord(ev[1], st);
    (void)hipEventRecord(ev[2], st);
    if (!fused) k_kick_drift<real><<<m->n_blocks, BS, 0, st>>>(C, 1);
    (void)hipEventRecord(ev[3], st);
    (void)hipEventRecord(ev[4], st);
    launch_bin<real>(m, C, m->n_boxes, st, fused ? 1 : -1);
    (void)hipEventRecord(ev[5], st);
    (void)hipEventRecord(ev[6], st);
    launch_forces<real>(m, C, m->n_blocks, 1, 1, st);
    (void)hipEventRecord(ev[7], st);
    (void)hipEventRecord(ev[8], st);  // the second half kick runs inside the force kernel
    (void)hipEventRecord(ev[9], st);
    (void)hipEventRecord(ev[10], st);
    k_box_stress<<<m->n_boxes, 64, 0, st>>>(C);
    (void)hipEventRecord(ev[11], st);
}

// Copy the step counter *src to dst[0 .. n-1].
__global__ void k_step_copy(unsigned long long* __restrict__ dst, const unsigned long long* __restrict__ src, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = *src;
}

// A captured chunk of nsteps steps with the boxes in overlapped groups.  The
// boxes of one group never read another group's data, so each group runs
// its whole chunk (fused binning, forces, stress) on its own stream with its
// own copy of the step counter: a group with small boxes does not wait each
// step for the binning of the largest ones.  The counters fork from the
// engine's at the start and join into it at the end; every box computes
// exactly what the stepwise order computes.
template <typename real>
void launch_chunk_grouped(lhmm_micro* m, int nsteps) {
    const int G = (int)m->groups.size();
    k_step_copy<<<1, 64, 0, m->stream>>>(m->d_gstep, m->d_step, G);
    (void)hipEventRecord(m->ev_fork, m->stream);
    for (int g = 1; g < G; ++g) (void)hipStreamWaitEvent(m->aux[g - 1], m->ev_fork, 0);
    for (int g = 0; g < G; ++g) {
        const lhmm_micro::Group& gr = m->groups[g];
        hipStream_t st = g == 0 ? m->stream : m->aux[g - 1];
        Ctx C = m->ctx;
        C.sel = gr.d_sel;
        C.blk_list = gr.d_blk;
        C.n_sel = gr.n_sel;
        C.step = m->d_gstep + g;
        for (int k = 0; k < nsteps; ++k) {
            if (gr.n_chunks > 0) {
                const SplitArgs& S = gr.S;
                const size_t scan_lds = sizeof(int) * ((size_t)gr.lds_cells + 3 * (size_t)gr.lds_cols);
                k_cell_step<<<(gr.n_sel + 255) / 256, 256, 0, st>>>(C, 1);
                k_bin_count<real><<<gr.n_chunks, SPLIT_BT, sizeof(int) * (size_t)S.cap, st>>>(C, S);
                k_bin_scan<<<gr.n_sel, SPLIT_BT, scan_lds, st>>>(C, S, gr.lds_cells, gr.lds_cols);
                k_bin_scatter<real><<<gr.n_chunks, SPLIT_BT, sizeof(int) * ((size_t)S.cap + S.chunk), st>>>(C, S);
            } else {
                launch_bin<real>(m, C, gr.n_sel, st, 1, gr.lds_cells, gr.lds_cols, gr.lds_parts);
            }
            launch_forces<real>(m, C, gr.nblk, 1, 1, st);
            k_box_stress<<<gr.n_sel, 64, 0, st>>>(C);
        }
    }
    for (int g = 1; g < G; ++g) {
        (void)hipEventRecord(m->ev_join[g - 1], m->aux[g - 1]);
        (void)hipStreamWaitEvent(m->stream, m->ev_join[g - 1], 0);
    }
    k_step_copy<<<1, 64, 0, m->stream>>>(m->d_step, m->d_gstep, 1);
}

void launch_one_step(lhmm_micro* m) {
    if (m->precision == LHMM_FP64)
        launch_step_kernels<double>(m, m->ctx, m->n_boxes, m->n_blocks, 1, true, true);
    else
        launch_step_kernels<float>(m, m->ctx, m->n_boxes, m->n_blocks, 1, true, true);
}

void launch_one_step_sel(lhmm_micro* m, const Ctx& C, int nbox, int nblk) {
    if (m->precision == LHMM_FP64)
        launch_step_kernels<double>(m, C, nbox, nblk, 1, true, true);
    else
        launch_step_kernels<float>(m, C, nbox, nblk, 1, true, true);
}

void launch_remove_mean(lhmm_micro* m, const Ctx& C, int nbox) {
    if (m->precision == LHMM_FP64)
        k_remove_mean<double><<<nbox, 256, 0, m->stream>>>(C);
    else
        k_remove_mean<float><<<nbox, 256, 0, m->stream>>>(C);
}

void launch_force_eval(lhmm_micro* m) {
    if (m->precision == LHMM_FP64)
        launch_step_kernels<double>(m, m->ctx, m->n_boxes, m->n_blocks, 0, false, false);
    else
        launch_step_kernels<float>(m, m->ctx, m->n_boxes, m->n_blocks, 0, false, false);
}

int get_graph(lhmm_micro* m, int nsteps, hipGraphExec_t* out) {
    auto it = m->graphs.find(nsteps);
    if (it != m->graphs.end()) {
        *out = it->second;
        return LHMM_OK;
    }
    hipGraph_t g = nullptr;
    const bool grouped = m->groups.size() > 1 && m->cfg.fuse_bin;
    HIPCHK(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
    if (!grouped)
        for (int k = 0; k < nsteps; ++k) launch_one_step(m);
    else if (m->precision == LHMM_FP64)
        launch_chunk_grouped<double>(m, nsteps);
    else
        launch_chunk_grouped<float>(m, nsteps);
    HIPCHK(hipStreamEndCapture(m->stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LHMM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    m->graphs[nsteps] = ex;
    *out = ex;
    return LHMM_OK;
}

bool cell_ok(const double* h) {
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(h[k])) return false;
    if (h[2] != 0.0 || h[5] != 0.0 || h[6] != 0.0 || h[7] != 0.0) return false;
    if (!(h[8] > 0.0)) return false;
    return m3_det(h) > 0.0;
}

template <typename T>
int dalloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return fail(LHMM_ERR_OOM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
    return LHMM_OK;
}

void release(lhmm_micro* m) {
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (auto& kv : m->graphs) (void)hipGraphExecDestroy(kv.second);
    m->graphs.clear();
    for (auto& kv : m->sub_graphs) (void)hipGraphExecDestroy(kv.second);
    m->sub_graphs.clear();
    void* bufs[] = {m->d_box, m->d_dyn, m->d_flags, m->d_blk_box, m->d_blk_first, m->d_s, m->d_c, m->d_f,
                    m->d_pcell, m->d_cell_start, m->d_gcell_start, m->d_cell_pv, m->d_srec,
                    m->d_part_vir, m->d_part_kin,
                    m->d_part_pairs, m->d_acc, m->d_parts, m->d_gradL, m->d_acc_pairs, m->d_tot_pairs, m->d_step, m->d_gstep,
                    m->d_sel, m->d_blk_list, m->d_snap_s, m->d_snap_c, m->d_snap_f, m->d_snap_dyn};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& gr : m->groups) {
        if (gr.d_sel) (void)hipFree(gr.d_sel);
        if (gr.d_blk) (void)hipFree(gr.d_blk);
        if (gr.d_split) (void)hipFree(gr.d_split);
    }
    m->groups.clear();
    for (int g = 0; g < MAX_GROUPS - 1; ++g) {
        if (m->aux[g]) (void)hipStreamDestroy(m->aux[g]);
        if (m->ev_join[g]) (void)hipEventDestroy(m->ev_join[g]);
    }
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->h_sel) (void)hipHostFree(m->h_sel);
    if (m->ev_sel) (void)hipEventDestroy(m->ev_sel);
    if (m->ev_in) (void)hipEventDestroy(m->ev_in);
    if (m->ev_out) (void)hipEventDestroy(m->ev_out);
    if (m->stream) (void)hipStreamDestroy(m->stream);
}

int sync_engine(lhmm_micro* m) {
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipGetLastError());
    return LHMM_OK;
}

constexpr size_t MAX_SUB_GRAPHS = 64;

// len steps of the selected boxes: a captured graph for a shape seen before,
// else eager launches.  The graph reads the selection lists from the fixed
// device buffers, so any selection of the same shape can replay it.
int launch_subset_steps(lhmm_micro* m, const Ctx& C, int n_sel, int nblk, int len) {
    const auto key = std::make_tuple(n_sel, nblk, len);
    auto it = m->sub_graphs.find(key);
    if (it == m->sub_graphs.end() && ++m->sub_seen[key] >= 2) {
        if (m->sub_graphs.size() >= MAX_SUB_GRAPHS) {
            for (auto& kv : m->sub_graphs) (void)hipGraphExecDestroy(kv.second);
            m->sub_graphs.clear();
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < len; ++k) launch_one_step_sel(m, C, n_sel, nblk);
        HIPCHK(hipStreamEndCapture(m->stream, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LHMM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        it = m->sub_graphs.emplace(key, ex).first;
    }
    if (it != m->sub_graphs.end()) {
        HIPCHK(hipGraphLaunch(it->second, m->stream));
    } else {
        for (int k = 0; k < len; ++k) launch_one_step_sel(m, C, n_sel, nblk);
    }
    return LHMM_OK;
}

// Partition the boxes into G groups by particle count (smallest first), with
// their block lists and binning LDS.
int prepare_groups(lhmm_micro* m, int G) {
    HIPCHK(hipStreamSynchronize(m->stream));
    for (auto& gr : m->groups) {
        if (gr.d_sel) (void)hipFree(gr.d_sel);
        if (gr.d_blk) (void)hipFree(gr.d_blk);
        if (gr.d_split) (void)hipFree(gr.d_split);
    }
    m->groups.clear();
    if (G <= 1) return LHMM_OK;
    if (!m->ev_fork) {
        HIPCHK(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
        for (int g = 0; g < MAX_GROUPS - 1; ++g) {
            HIPCHK(hipStreamCreateWithFlags(&m->aux[g], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&m->ev_join[g], hipEventDisableTiming));
        }
    }
    std::vector<int> order(m->n_boxes);
    for (int b = 0; b < m->n_boxes; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m->box[a].n < m->box[b].n; });
    // the largest boxes, two thirds of the particles, form the last group
    // (their binning is the longest; measured best on uneven batches), the
    // rest is shared equally by the others
    std::vector<std::vector<int>> members(G);
    long long acc = 0;
    const long long third = std::max(1LL, m->n_total / 3);
    for (int b : order) {
        const int g = acc >= third ? G - 1 : (int)(acc * (G - 1) / third);
        members[std::min(g, G - 1)].push_back(b);
        acc += m->box[b].n;
    }
    for (int g = 0; g < G; ++g) {
        if (members[g].empty()) continue;
        std::sort(members[g].begin(), members[g].end());
        lhmm_micro::Group gr;
        std::vector<int> blks;
        int max_cells = 0, max_cols = 0, max_n = 0;
        for (int b : members[g]) {
            const BoxInfo& B = m->box[b];
            for (int k = 0; k < B.nblk; ++k) blks.push_back(B.blk_off + k);
            max_cells = std::max(max_cells, B.cell_cap + 1);
            max_cols = std::max(max_cols, box_cols(B));
            max_n = std::max(max_n, B.n);
        }
        gr.n_sel = (int)members[g].size();
        gr.nblk = (int)blks.size();
        gr.lds_cells = max_cells;
        gr.lds_cols = max_cols;
        const int fixed = max_cells + 3 * max_cols;
        const int room = m->bin_lds_cells + 3 * m->bin_lds_cols + m->bin_lds_parts - fixed;
        gr.lds_parts = std::max(0, std::min(max_n, room));
        int rc = dalloc(&gr.d_sel, gr.n_sel);
        if (rc == LHMM_OK) rc = dalloc(&gr.d_blk, gr.nblk);
        if (rc != LHMM_OK) {
            if (gr.d_sel) (void)hipFree(gr.d_sel);
            return rc;
        }
        if (g == G - 1 && m->cfg.bin_split > 0) {
            // chunks of the largest boxes for the split binning
            const int chunk = m->cfg.bin_split;
            std::vector<int> box_chunk0(gr.n_sel + 1, 0), chunk_boxj;
            for (int q = 0; q < gr.n_sel; ++q) {
                const int nck = std::max(1, (m->box[members[g][q]].n + chunk - 1) / chunk);
                box_chunk0[q + 1] = box_chunk0[q] + nck;
                for (int c = 0; c < nck; ++c) chunk_boxj.push_back(q);
            }
            gr.n_chunks = box_chunk0[gr.n_sel];
            const int cap = max_cells, colcap = max_cols;
            const size_t ints = (size_t)(gr.n_sel + 1) + gr.n_chunks + 2 * (size_t)gr.n_chunks * cap +
                                3 * (size_t)gr.n_sel * colcap;
            rc = dalloc(&gr.d_split, ints);
            if (rc != LHMM_OK) {
                (void)hipFree(gr.d_sel);
                (void)hipFree(gr.d_blk);
                return rc;
            }
            int* base = gr.d_split;
            gr.S.box_chunk0 = base;
            gr.S.chunk_boxj = base + gr.n_sel + 1;
            gr.S.cnt = base + gr.n_sel + 1 + gr.n_chunks;
            gr.S.off = gr.S.cnt + (size_t)gr.n_chunks * cap;
            gr.S.col = gr.S.off + (size_t)gr.n_chunks * cap;
            gr.S.chunk = chunk;
            gr.S.cap = cap;
            gr.S.colcap = colcap;
            HIPCHK(hipMemcpy(base, box_chunk0.data(), sizeof(int) * box_chunk0.size(), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(base + gr.n_sel + 1, chunk_boxj.data(), sizeof(int) * chunk_boxj.size(),
                             hipMemcpyHostToDevice));
        }
        m->groups.push_back(gr);
        HIPCHK(hipMemcpy(gr.d_sel, members[g].data(), sizeof(int) * gr.n_sel, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(gr.d_blk, blks.data(), sizeof(int) * gr.nblk, hipMemcpyHostToDevice));
    }
    return LHMM_OK;
}

// Validate a host list of boxes (strictly increasing, in range), upload it
// and the list of their work blocks on the engine stream, and return a
// context that selects them.
int select_boxes(lhmm_micro* m, const int32_t* boxes, int32_t n_sel, Ctx* out, int* nblk) {
    if (!boxes || n_sel < 1 || n_sel > m->n_boxes) return fail(LHMM_ERR_ARG, "need 1..%d boxes (got %d)", m->n_boxes, n_sel);
    for (int q = 0; q < n_sel; ++q) {
        if (boxes[q] < 0 || boxes[q] >= m->n_boxes) return fail(LHMM_ERR_ARG, "box %d out of range", boxes[q]);
        if (q && boxes[q] <= boxes[q - 1]) return fail(LHMM_ERR_ARG, "boxes must be strictly increasing");
    }
    if (!m->d_sel) {
        int rc = dalloc(&m->d_sel, m->n_boxes);
        if (rc == LHMM_OK) rc = dalloc(&m->d_blk_list, m->n_blocks);
        if (rc != LHMM_OK) return rc;
        HIPCHK(hipHostMalloc((void**)&m->h_sel, sizeof(int) * (m->n_boxes + m->n_blocks)));
        HIPCHK(hipEventCreateWithFlags(&m->ev_sel, hipEventDisableTiming));
    } else {
        HIPCHK(hipEventSynchronize(m->ev_sel));  // the previous upload has left the staging buffer
    }
    int nb = 0;
    int* hb = m->h_sel + m->n_boxes;
    for (int q = 0; q < n_sel; ++q) {
        const BoxInfo& B = m->box[boxes[q]];
        m->h_sel[q] = boxes[q];
        for (int k = 0; k < B.nblk; ++k) hb[nb++] = B.blk_off + k;
    }
    HIPCHK(hipMemcpyAsync(m->d_sel, m->h_sel, sizeof(int) * n_sel, hipMemcpyHostToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->d_blk_list, hb, sizeof(int) * nb, hipMemcpyHostToDevice, m->stream));
    HIPCHK(hipEventRecord(m->ev_sel, m->stream));
    *out = m->ctx;
    out->sel = m->d_sel;
    out->blk_list = m->d_blk_list;
    out->n_sel = n_sel;
    *nblk = nb;
    return LHMM_OK;
}

}  // namespace

int lhmm_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void lhmm_clear_error() { g_err.clear(); }

hipStream_t lhmm_micro_caller_stream(const lhmm_micro* m) { return m->user_stream; }

extern "C" {

const char* lhmm_last_error(void) { return g_err.c_str(); }

int lhmm_micro_create(const lhmm_params* p, const lhmm_box* boxes, int32_t n_boxes, void* stream,
                      lhmm_micro** out) {
    g_err.clear();
    if (!p || !boxes || !out) return fail(LHMM_ERR_ARG, "null argument");
    *out = nullptr;
    if (n_boxes <= 0) return fail(LHMM_ERR_ARG, "n_boxes must be positive (got %d)", n_boxes);
    const double vals[9] = {p->a, p->gamma, p->sigma, p->kBT, p->mass, p->rc, p->dt, p->H, p->R0};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(LHMM_ERR_ARG, "non-finite parameter");
    if (!(p->dt > 0) || !(p->rc > 0) || !(p->mass > 0) || !(p->R0 > 0) || p->gamma < 0 || p->sigma < 0 || p->H < 0)
        return fail(LHMM_ERR_ARG, "parameters out of range (dt, rc, mass, R0 > 0; gamma, sigma, H >= 0)");
    if (p->chain_len < 2) return fail(LHMM_ERR_ARG, "chain_len must be >= 2");
    if (p->precision != LHMM_FP32 && p->precision != LHMM_FP64) return fail(LHMM_ERR_ARG, "bad precision");

    lhmm_micro* m = new (std::nothrow) lhmm_micro();
    if (!m) return fail(LHMM_ERR_OOM, "host allocation failed");
    m->p = *p;
    m->n_boxes = n_boxes;
    m->precision = p->precision;
    m->cfg.queue_depth = 16;
    m->cfg.drain = 12;
    m->cfg.busy_lanes = 65;
    m->cfg.bin_threads = BIN_THREADS_MAX;
    m->cfg.graph_chunk = GRAPH_CHUNK;
    m->cfg.prune = 0;
    m->cfg.fuse_bin = 1;
    m->cfg.groups = 2;
    m->cfg.bin_split = 0;
    m->real_size = p->precision == LHMM_FP64 ? sizeof(double) : sizeof(float);
    m->user_stream = (hipStream_t)stream;

    long long off = 0;
    int cell_off = 0, gcell_off = 0, blk_off = 0;
    m->box.resize(n_boxes);
    for (int b = 0; b < n_boxes; ++b) {
        const lhmm_box& in = boxes[b];
        if (in.n_particles < 2 || in.n_particles > (1 << 25) || in.n_chains < 0 ||
            (long long)in.n_chains * p->chain_len > in.n_particles) {
            delete m;
            return fail(LHMM_ERR_ARG, "box %d: bad particle/chain counts", b);
        }
        if (in.reserved != 0) {
            delete m;
            return fail(LHMM_ERR_ARG, "box %d: reserved field must be 0", b);
        }
        if (!cell_ok(in.h0)) {
            delete m;
            return fail(LHMM_ERR_ARG, "box %d: cell must be finite, in-plane, with det > 0", b);
        }
        // n0 n1 <= w0 w1 <= area and n2 = floor(zsub z extent / rc): the grid
        // never needs more; two cells per cutoff along z unless that exceeds
        // the cell limit
        const double area = fabs(in.h0[0] * in.h0[4] - in.h0[1] * in.h0[3]);
        const long long inplane = (long long)std::floor(area / (p->rc * p->rc) * (1.0 + 1e-9));
        long long cap = 0;
        int zsub = 2;
        for (; zsub >= 1; --zsub) {
            const long long nz = (long long)std::floor(zsub * in.h0[8] / p->rc * (1.0 + 1e-9));
            cap = std::max(9LL * (2 * zsub + 1), std::max(inplane, 9LL) * std::max(nz, 2LL * zsub + 1));
            if (cap <= MAX_CELLS_PER_BOX) break;
        }
        if (cap > MAX_CELLS_PER_BOX) {
            delete m;
            return fail(LHMM_ERR_ARG, "box %d: needs %lld cells, more than %d", b, cap, MAX_CELLS_PER_BOX);
        }
        BoxInfo& B = m->box[b];
        B.off = (int)off;
        B.n = in.n_particles;
        B.n_beads = in.n_chains * p->chain_len;
        B.cell_off = cell_off;
        B.cell_cap = (int)cap;
        B.gcell_off = gcell_off;
        B.zsub = zsub;
        B.blk_off = blk_off;
        B.nblk = (in.n_particles + BS - 1) / BS;
        B.rng_id = in.rng_id;
        for (int k = 0; k < B.nblk; ++k) {
            m->blk_box.push_back(b);
            m->blk_first.push_back(B.off + k * BS);
        }
        off += in.n_particles;
        cell_off += (int)cap + 1;
        gcell_off += 2 * (int)cap + 1;  // n0 n1 (n2 + 2 zsub) cells, n2 >= 2 zsub + 1
        blk_off += B.nblk;
        if (off > (1LL << 30)) {
            delete m;
            return fail(LHMM_ERR_ARG, "too many particles");
        }
    }
    m->n_total = off;
    m->n_blocks = blk_off;
    {
        // binning LDS: three arrays over every box's cells, and entries for
        // the boxes that fit in what the workgroup may still use
        int max_cells = 0, max_cols = 0, max_n = 0;
        for (const BoxInfo& B : m->box) {
            max_cells = std::max(max_cells, B.cell_cap + 1);
            max_cols = std::max(max_cols, box_cols(B));
            max_n = std::max(max_n, B.n);
        }
        int dev = 0, max_lds = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            max_lds = 65536;
        const int budget = (int)((max_lds - 64 * (int)sizeof(int)) / sizeof(int));  // less the scan's wave sums
        const int fixed = max_cells + 3 * max_cols;  // cells and column offsets
        if (fixed > budget) {
            delete m;
            return fail(LHMM_ERR_ARG, "boxes need %d cells, more than the binning LDS holds", max_cells - 1);
        }
        m->bin_lds_cells = max_cells;
        m->bin_lds_cols = max_cols;
        m->bin_lds_parts = std::max(0, std::min(max_n, budget - fixed));
        const size_t bytes = sizeof(int) * ((size_t)fixed + (size_t)m->bin_lds_parts);
        const void* kernels[] = {(const void*)&k_bin_box<float, 256>, (const void*)&k_bin_box<float, 512>,
                                 (const void*)&k_bin_box<float, 1024>, (const void*)&k_bin_box<double, 256>,
                                 (const void*)&k_bin_box<double, 512>, (const void*)&k_bin_box<double, 1024>};
        for (const void* k : kernels) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) {
                delete m;
                return fail(LHMM_ERR_HIP, "binning LDS of %zu bytes: %s", bytes, hipGetErrorString(e));
            }
        }
        // split binning: cells + column offsets (scan), cells + a chunk (scatter), cells (count)
        const size_t split_bytes[] = {sizeof(int) * (size_t)fixed, sizeof(int) * ((size_t)max_cells + SPLIT_PER * SPLIT_BT),
                                      sizeof(int) * (size_t)max_cells};
        const void* split_kernels[][2] = {{(const void*)&k_bin_scan, (const void*)&k_bin_scan},
                                          {(const void*)&k_bin_scatter<float>, (const void*)&k_bin_scatter<double>},
                                          {(const void*)&k_bin_count<float>, (const void*)&k_bin_count<double>}};
        for (int q = 0; q < 3; ++q)
            for (const void* k : split_kernels[q]) {
                hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)split_bytes[q]);
                if (e != hipSuccess) {
                    delete m;
                    return fail(LHMM_ERR_HIP, "split binning LDS of %zu bytes: %s", split_bytes[q], hipGetErrorString(e));
                }
            }
    }
    const size_t N = (size_t)m->n_total;
    int rc = LHMM_OK;
#define ALLOC(ptr, cnt)                     \
    if (rc == LHMM_OK) rc = dalloc(&(ptr), (cnt));
    ALLOC(m->d_box, (size_t)n_boxes);
    ALLOC(m->d_dyn, (size_t)n_boxes);
    ALLOC(m->d_flags, (size_t)n_boxes);
    ALLOC(m->d_blk_box, (size_t)m->n_blocks);
    ALLOC(m->d_blk_first, (size_t)m->n_blocks);
    ALLOC(m->d_pcell, N);
    ALLOC(m->d_cell_start, (size_t)cell_off);
    ALLOC(m->d_gcell_start, (size_t)gcell_off);
    const int pv_stride = (p->flags & LHMM_OPT_COMPONENTS) ? 30 : 12;
    ALLOC(m->d_part_vir, (size_t)m->n_blocks * pv_stride);
    ALLOC(m->d_part_kin, (size_t)m->n_blocks * 6);
    ALLOC(m->d_part_pairs, (size_t)m->n_blocks);
    ALLOC(m->d_acc, (size_t)n_boxes * ACC);
    ALLOC(m->d_parts, (size_t)n_boxes * ACC);
    ALLOC(m->d_gradL, (size_t)n_boxes * 9);
    ALLOC(m->d_acc_pairs, (size_t)n_boxes);
    ALLOC(m->d_tot_pairs, (size_t)n_boxes);
    ALLOC(m->d_step, (size_t)1);
    ALLOC(m->d_gstep, (size_t)MAX_GROUPS);
#undef ALLOC
    if (rc == LHMM_OK) {
        const size_t bytes = 3 * N * m->real_size;
        // search layout: each particle at most twice (its cell, and the
        // image of a bottom or top cell; n2 >= 3)
        for (void** pp : {&m->d_s, &m->d_c, &m->d_f, &m->d_cell_pv, &m->d_srec}) {
            const size_t nb = pp == &m->d_cell_pv ? 8 * N * m->real_size
                              : pp == &m->d_srec ? (8 * N + 16) * m->real_size : bytes;
            if (hipMalloc(pp, nb ? nb : 1) != hipSuccess) {
                rc = fail(LHMM_ERR_OOM, "hipMalloc of particle arrays failed");
                break;
            }
        }
    }
    if (rc != LHMM_OK) {
        release(m);
        delete m;
        return rc;
    }
    auto setup = [&]() -> int {
        HIPCHK(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
        HIPCHK(hipMemcpy(m->d_box, m->box.data(), n_boxes * sizeof(BoxInfo), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->d_blk_box, m->blk_box.data(), m->n_blocks * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->d_blk_first, m->blk_first.data(), m->n_blocks * sizeof(int), hipMemcpyHostToDevice));
        std::vector<BoxDyn> dyn(n_boxes);
        for (int b = 0; b < n_boxes; ++b) {
            memset(&dyn[b], 0, sizeof(BoxDyn));
            for (int k = 0; k < 9; ++k) dyn[b].h[k] = boxes[b].h0[k];
        }
        HIPCHK(hipMemcpy(m->d_dyn, dyn.data(), n_boxes * sizeof(BoxDyn), hipMemcpyHostToDevice));
        HIPCHK(hipMemset(m->d_flags, 0, n_boxes * sizeof(unsigned)));
        HIPCHK(hipMemset(m->d_acc, 0, n_boxes * ACC * sizeof(double)));
        HIPCHK(hipMemset(m->d_parts, 0, n_boxes * ACC * sizeof(double)));
        HIPCHK(hipMemset(m->d_acc_pairs, 0, n_boxes * sizeof(unsigned long long)));
        HIPCHK(hipMemset(m->d_tot_pairs, 0, n_boxes * sizeof(unsigned long long)));
        HIPCHK(hipMemset(m->d_step, 0, sizeof(unsigned long long)));
        if (N) HIPCHK(hipMemset(m->d_f, 0, 3 * N * m->real_size));
        return LHMM_OK;
    };
    rc = setup();
    if (rc != LHMM_OK) {
        release(m);
        delete m;
        return rc;
    }
    Ctx& C = m->ctx;
    C.n_total = (int)m->n_total;
    C.n_boxes = n_boxes;
    C.n_blocks = m->n_blocks;
    C.chain_len = p->chain_len;
    C.box = m->d_box;
    C.dyn = m->d_dyn;
    C.flags = m->d_flags;
    C.blk_box = m->d_blk_box;
    C.blk_first = m->d_blk_first;
    C.s = m->d_s;
    C.c = m->d_c;
    C.f = m->d_f;
    C.pcell = m->d_pcell;
    C.cell_start = m->d_cell_start;
    C.gcell_start = m->d_gcell_start;
    C.cell_pv = m->d_cell_pv;
    C.srec = m->d_srec;
    C.vir_scale = 0.5;  // every unordered pair is evaluated from both ends
    C.part_vir = m->d_part_vir;
    C.pv_stride = pv_stride;
    C.part_kin = m->d_part_kin;
    C.part_pairs = m->d_part_pairs;
    C.acc = m->d_acc;
    C.acc_pairs = m->d_acc_pairs;
    C.tot_pairs = m->d_tot_pairs;
    C.step = m->d_step;
    C.a = p->a;
    C.gamma = p->gamma;
    C.sigma = p->sigma;
    C.rdt = 1.0 / std::sqrt(p->dt);
    C.dt = p->dt;
    C.mass = p->mass;
    C.inv_mass = 1.0 / p->mass;
    C.rc = p->rc;
    C.rc2 = p->rc * p->rc;
    C.H = p->H;
    C.inv_R02 = 1.0 / (p->R0 * p->R0);
    C.key0 = (unsigned)(p->seed & 0xFFFFFFFFull);
    C.key1 = (unsigned)(p->seed >> 32);
    rc = prepare_groups(m, m->cfg.groups);
    if (rc != LHMM_OK) {
        release(m);
        delete m;
        return rc;
    }
    *out = m;
    return LHMM_OK;
}

int lhmm_micro_set_state(lhmm_micro* m, const double* s, const double* c, const double* f, const double* h,
                         uint64_t step) {
    g_err.clear();
    if (!m || !s || !c) return fail(LHMM_ERR_ARG, "null argument");
    const size_t N = (size_t)m->n_total;
    for (size_t k = 0; k < 3 * N; ++k) {
        if (!(s[k] >= 0.0 && s[k] < 1.0)) return fail(LHMM_ERR_ARG, "s[%zu] = %g outside [0, 1)", k, s[k]);
        if (!std::isfinite(c[k])) return fail(LHMM_ERR_ARG, "c[%zu] is not finite", k);
        if (f && !std::isfinite(f[k])) return fail(LHMM_ERR_ARG, "f[%zu] is not finite", k);
    }
    if (h)
        for (int b = 0; b < m->n_boxes; ++b)
            if (!cell_ok(h + 9 * b)) return fail(LHMM_ERR_ARG, "box %d: bad cell", b);
    HIPCHK(hipStreamSynchronize(m->stream));
    // AoS double -> SoA real
    std::vector<char> buf(3 * N * m->real_size + 1);
    const double* srcs[3] = {s, c, f};
    void* dsts[3] = {m->d_s, m->d_c, m->d_f};
    for (int which = 0; which < 3; ++which) {
        const double* src = srcs[which];
        if (!src) continue;
        for (size_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                const double v = src[3 * i + k];
                if (m->precision == LHMM_FP64) {
                    ((double*)buf.data())[k * N + i] = v;
                } else {
                    float x = (float)v;
                    if (which == 0 && x >= 1.0f) x = 0.0f;
                    ((float*)buf.data())[k * N + i] = x;
                }
            }
        HIPCHK(hipMemcpy(dsts[which], buf.data(), 3 * N * m->real_size, hipMemcpyHostToDevice));
    }
    if (h) {
        std::vector<BoxDyn> dyn(m->n_boxes);
        HIPCHK(hipMemcpy(dyn.data(), m->d_dyn, m->n_boxes * sizeof(BoxDyn), hipMemcpyDeviceToHost));
        for (int b = 0; b < m->n_boxes; ++b)
            for (int k = 0; k < 9; ++k) dyn[b].h[k] = h[9 * b + k];
        HIPCHK(hipMemcpy(m->d_dyn, dyn.data(), m->n_boxes * sizeof(BoxDyn), hipMemcpyHostToDevice));
    }
    unsigned long long st = step;
    HIPCHK(hipMemcpy(m->d_step, &st, sizeof st, hipMemcpyHostToDevice));
    m->have_state = true;
    m->forces_valid = f != nullptr;
    return LHMM_OK;
}

int lhmm_micro_get_state(lhmm_micro* m, double* s, double* c, double* f, double* h, uint64_t* step) {
    g_err.clear();
    if (!m) return fail(LHMM_ERR_ARG, "null engine");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    const size_t N = (size_t)m->n_total;
    std::vector<char> buf(3 * N * m->real_size + 1);
    double* dsts[3] = {s, c, f};
    const void* srcs[3] = {m->d_s, m->d_c, m->d_f};
    for (int which = 0; which < 3; ++which) {
        double* dst = dsts[which];
        if (!dst) continue;
        HIPCHK(hipMemcpy(buf.data(), srcs[which], 3 * N * m->real_size, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k)
                dst[3 * i + k] = m->precision == LHMM_FP64 ? ((double*)buf.data())[k * N + i]
                                                           : (double)((float*)buf.data())[k * N + i];
    }
    if (h) {
        std::vector<BoxDyn> dyn(m->n_boxes);
        HIPCHK(hipMemcpy(dyn.data(), m->d_dyn, m->n_boxes * sizeof(BoxDyn), hipMemcpyDeviceToHost));
        for (int b = 0; b < m->n_boxes; ++b)
            for (int k = 0; k < 9; ++k) h[9 * b + k] = dyn[b].h[k];
    }
    if (step) {
        unsigned long long st = 0;
        HIPCHK(hipMemcpy(&st, m->d_step, sizeof st, hipMemcpyDeviceToHost));
        *step = st;
    }
    return LHMM_OK;
}

int lhmm_micro_step(lhmm_micro* m, const double* gradL, int32_t n_steps, double* stress_out) {
    g_err.clear();
    if (!m || !gradL || !stress_out) return fail(LHMM_ERR_ARG, "null argument");
    if (n_steps <= 0) return fail(LHMM_ERR_ARG, "n_steps must be positive (got %d)", n_steps);
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    const int bt = 256, bg = (m->n_boxes + bt - 1) / bt;
    HIPCHK(hipEventRecord(m->ev_in, m->user_stream));
    HIPCHK(hipStreamWaitEvent(m->stream, m->ev_in, 0));
    k_setup_call<<<bg, bt, 0, m->stream>>>(m->ctx, gradL);
    k_zero_acc<<<(ACC * m->n_boxes + 255) / 256, 256, 0, m->stream>>>(m->ctx);
    launch_remove_mean(m, m->ctx, m->n_boxes);
    if (!m->forces_valid) {
        launch_force_eval(m);
        m->forces_valid = true;
    }
    HIPCHK(hipGetLastError());
    if (m->p.flags & LHMM_OPT_NO_GRAPH) {
        for (int k = 0; k < n_steps; ++k) launch_one_step(m);
    } else {
        const int chunk = n_steps < m->cfg.graph_chunk ? n_steps : m->cfg.graph_chunk;
        const int full = n_steps / chunk, rest = n_steps % chunk;
        hipGraphExec_t g = nullptr;
        int rc = get_graph(m, chunk, &g);
        if (rc != LHMM_OK) return rc;
        for (int k = 0; k < full; ++k) HIPCHK(hipGraphLaunch(g, m->stream));
        if (rest) {
            rc = get_graph(m, rest, &g);
            if (rc != LHMM_OK) return rc;
            HIPCHK(hipGraphLaunch(g, m->stream));
        }
    }
    k_finalize<<<bg, bt, 0, m->stream>>>(m->ctx, stress_out, m->d_parts, 1.0 / n_steps);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(m->ev_out, m->stream));
    HIPCHK(hipStreamWaitEvent(m->user_stream, m->ev_out, 0));
    return LHMM_OK;
}

int lhmm_micro_set_config(lhmm_micro* m, const lhmm_micro_config* cfg) {
    g_err.clear();
    if (!m || !cfg) return fail(LHMM_ERR_ARG, "null argument");
    const int qd = cfg->queue_depth;
    const bool qd_ok = qd == 2 || qd == 4 || qd == 8 || qd == 16 || qd == 32;
    if (!qd_ok) return fail(LHMM_ERR_ARG, "queue_depth must be 2, 4, 8, 16 or 32");
    // a search iteration pushes up to scan_unroll(qd) neighbours per lane
    // before it checks the queues, so a lane may hold at most qd - that many
    // when the search resumes
    const int dmax = qd - scan_unroll(qd);
    if (cfg->drain < 0 || cfg->drain > dmax) return fail(LHMM_ERR_ARG, "drain must be in 0..%d", dmax);
    if (cfg->busy_lanes < 1 || cfg->busy_lanes > 65) return fail(LHMM_ERR_ARG, "busy_lanes must be in 1..65");
    if (cfg->bin_threads != 256 && cfg->bin_threads != 512 && cfg->bin_threads != 1024)
        return fail(LHMM_ERR_ARG, "bin_threads must be 256, 512 or 1024");
    if (cfg->graph_chunk < 1 || cfg->graph_chunk > 1000) return fail(LHMM_ERR_ARG, "graph_chunk must be 1..1000");
    if (cfg->prune != 0 && cfg->prune != 1) return fail(LHMM_ERR_ARG, "prune must be 0 or 1");
    if (cfg->fuse_bin != 0 && cfg->fuse_bin != 1) return fail(LHMM_ERR_ARG, "fuse_bin must be 0 or 1");
    if (cfg->groups < 1 || cfg->groups > MAX_GROUPS) return fail(LHMM_ERR_ARG, "groups must be 1..%d", MAX_GROUPS);
    if (cfg->bin_split != 0 && (cfg->bin_split < 256 || cfg->bin_split > SPLIT_PER * SPLIT_BT))
        return fail(LHMM_ERR_ARG, "bin_split must be 0 or 256..%d", SPLIT_PER * SPLIT_BT);
    HIPCHK(hipStreamSynchronize(m->stream));
    for (auto& kv : m->graphs) (void)hipGraphExecDestroy(kv.second);
    m->graphs.clear();
    for (auto& kv : m->sub_graphs) (void)hipGraphExecDestroy(kv.second);
    m->sub_graphs.clear();
    m->sub_seen.clear();
    const bool regroup = cfg->groups != m->cfg.groups || cfg->bin_split != m->cfg.bin_split;
    m->cfg = *cfg;
    return regroup ? prepare_groups(m, cfg->groups) : LHMM_OK;
}

int lhmm_micro_set_afbc(lhmm_micro* m, const double* regions, double zeta) {
    g_err.clear();
    if (!m || !regions) return fail(LHMM_ERR_ARG, "null argument");
    if (!(zeta >= 0.0) || !std::isfinite(zeta)) return fail(LHMM_ERR_ARG, "zeta must be finite and >= 0");
    HIPCHK(hipStreamSynchronize(m->stream));
    std::vector<BoxDyn> dyn(m->n_boxes);
    HIPCHK(hipMemcpy(dyn.data(), m->d_dyn, m->n_boxes * sizeof(BoxDyn), hipMemcpyDeviceToHost));
    bool any = false;
    for (int b = 0; b < m->n_boxes; ++b) {
        const double hc = regions[2 * b], hb = regions[2 * b + 1];
        if (hc == 0.0 && hb == 0.0) continue;
        double w[3];
        m3_widths(dyn[b].h, w);
        if (!(hc > 0.0) || !(hb >= hc) || !(hb <= 0.5 * std::min(w[0], w[1])) || !std::isfinite(hb))
            return fail(LHMM_ERR_ARG, "box %d: need 0 < hc <= hb <= half the cell's in-plane width (%g)", b,
                        0.5 * std::min(w[0], w[1]));
        any = true;
    }
    for (int b = 0; b < m->n_boxes; ++b) {
        dyn[b].hc = regions[2 * b];
        dyn[b].hb = regions[2 * b + 1];
        if (dyn[b].hc == 0.0)
            for (int k = 0; k < 4; ++k) dyn[b].G[k] = 0.0;
    }
    HIPCHK(hipMemcpy(m->d_dyn, dyn.data(), m->n_boxes * sizeof(BoxDyn), hipMemcpyHostToDevice));
    m->afbc = any;
    const double dt = m->p.dt;
    m->ctx.ou_damp = std::exp(-0.5 * zeta * dt);
    m->ctx.ou_amp = std::sqrt(m->p.kBT / m->p.mass * (1.0 - std::exp(-zeta * dt)));
    // captured graphs hold the kernel variant and the context
    for (auto& kv : m->graphs) (void)hipGraphExecDestroy(kv.second);
    m->graphs.clear();
    for (auto& kv : m->sub_graphs) (void)hipGraphExecDestroy(kv.second);
    m->sub_graphs.clear();
    m->sub_seen.clear();
    return LHMM_OK;
}

int lhmm_micro_get_config(lhmm_micro* m, lhmm_micro_config* cfg) {
    g_err.clear();
    if (!m || !cfg) return fail(LHMM_ERR_ARG, "null argument");
    *cfg = m->cfg;
    return LHMM_OK;
}

int lhmm_micro_autotune(lhmm_micro* m, const double* gradL, int32_t trial_steps, lhmm_micro_config* best,
                        double* best_ms) {
    g_err.clear();
    if (!m || !gradL) return fail(LHMM_ERR_ARG, "null argument");
    if (trial_steps < 1) return fail(LHMM_ERR_ARG, "trial_steps must be positive");
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    // keep the state (particles, cells, counter, flags) to put it back after every trial
    const size_t bytes = 3 * (size_t)m->n_total * m->real_size;
    void *ss = nullptr, *sc = nullptr, *sf = nullptr, *sdyn = nullptr, *sflags = nullptr, *sout = nullptr;
    unsigned long long step0 = 0;
    int rc = dalloc((char**)&ss, bytes);
    if (rc == LHMM_OK) rc = dalloc((char**)&sc, bytes);
    if (rc == LHMM_OK) rc = dalloc((char**)&sf, bytes);
    if (rc == LHMM_OK) rc = dalloc((char**)&sdyn, sizeof(BoxDyn) * m->n_boxes);
    if (rc == LHMM_OK) rc = dalloc((char**)&sflags, sizeof(unsigned) * m->n_boxes);
    if (rc == LHMM_OK) rc = dalloc((char**)&sout, sizeof(double) * 6 * m->n_boxes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(m->stream);
        for (void* q : {ss, sc, sf, sdyn, sflags, sout})
            if (q) (void)hipFree(q);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return code;
    };
    if (rc != LHMM_OK) return done(rc);
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return done(fail(LHMM_ERR_HIP, "hipEventCreate failed"));
    if (hipStreamSynchronize(m->user_stream) != hipSuccess || sync_engine(m) != LHMM_OK)
        return done(fail(LHMM_ERR_HIP, "synchronisation failed"));
    const bool fv = m->forces_valid;
    auto save = [&]() -> hipError_t {
        hipError_t e = hipMemcpy(ss, m->d_s, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(sc, m->d_c, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(sf, m->d_f, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(sdyn, m->d_dyn, sizeof(BoxDyn) * m->n_boxes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(sflags, m->d_flags, sizeof(unsigned) * m->n_boxes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(&step0, m->d_step, sizeof step0, hipMemcpyDeviceToHost);
        return e;
    };
    auto load = [&]() -> hipError_t {
        hipError_t e = hipStreamSynchronize(m->stream);
        if (e == hipSuccess) e = hipMemcpy(m->d_s, ss, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_c, sc, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_f, sf, bytes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_dyn, sdyn, sizeof(BoxDyn) * m->n_boxes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_flags, sflags, sizeof(unsigned) * m->n_boxes, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_step, &step0, sizeof step0, hipMemcpyHostToDevice);
        m->forces_valid = fv;
        return e;
    };
    if (save() != hipSuccess) return done(fail(LHMM_ERR_HIP, "state copy failed"));
    // mean ms per step of one configuration (one warm-up call, then one timed call)
    auto trial = [&](const lhmm_micro_config& c, double* ms) -> int {
        int r = lhmm_micro_set_config(m, &c);
        if (r != LHMM_OK) return r;
        r = lhmm_micro_step(m, gradL, trial_steps, (double*)sout);
        if (r != LHMM_OK) return r;
        HIPCHK(hipEventRecord(e0, m->user_stream));
        r = lhmm_micro_step(m, gradL, trial_steps, (double*)sout);
        if (r != LHMM_OK) return r;
        HIPCHK(hipEventRecord(e1, m->user_stream));
        HIPCHK(hipEventSynchronize(e1));
        float el = 0.0f;
        HIPCHK(hipEventElapsedTime(&el, e0, e1));
        *ms = el / trial_steps;
        return load() == hipSuccess ? LHMM_OK : fail(LHMM_ERR_HIP, "state restore failed");
    };
    // coordinate search: force-kernel queue, binning workgroup, pruning, graph chunk
    lhmm_micro_config cur = m->cfg;
    double cur_ms = 0.0;
    rc = trial(cur, &cur_ms);
    const int qds[] = {8, 16, 32};
    for (int iq = 0; rc == LHMM_OK && iq < 3; ++iq) {
        const int qd = qds[iq];
        // (drain, busy): full drain range / no busy rule, or rounds driven by busy lanes
        const int dmax = qd - scan_unroll(qd);
        const int cand[4][2] = {{dmax, 65}, {qd / 2 <= dmax ? qd / 2 : dmax, 65}, {dmax, 56}, {0, 65}};
        for (const auto& dc : cand) {
            lhmm_micro_config c = cur;
            c.queue_depth = qd;
            c.drain = dc[0];
            c.busy_lanes = dc[1];
            if (c.queue_depth == cur.queue_depth && c.drain == cur.drain && c.busy_lanes == cur.busy_lanes) continue;
            double ms = 0.0;
            rc = trial(c, &ms);
            if (rc != LHMM_OK) break;
            if (ms < cur_ms) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    for (int bt : {256, 512, 1024}) {
        if (rc != LHMM_OK || bt == cur.bin_threads) continue;
        lhmm_micro_config c = cur;
        c.bin_threads = bt;
        double ms = 0.0;
        rc = trial(c, &ms);
        if (rc == LHMM_OK && ms < cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    for (int fb : {0, 1}) {
        if (rc != LHMM_OK || fb == cur.fuse_bin) continue;
        lhmm_micro_config c = cur;
        c.fuse_bin = fb;
        double ms = 0.0;
        rc = trial(c, &ms);
        if (rc == LHMM_OK && ms < cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    for (int pr : {0, 1}) {
        if (rc != LHMM_OK || pr == cur.prune) continue;
        lhmm_micro_config c = cur;
        c.prune = pr;
        double ms = 0.0;
        rc = trial(c, &ms);
        if (rc == LHMM_OK && ms < cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    for (int gr : {1, 2, 3}) {
        if (rc != LHMM_OK || gr == cur.groups) continue;
        lhmm_micro_config c = cur;
        c.groups = gr;
        double ms = 0.0;
        rc = trial(c, &ms);
        if (rc == LHMM_OK && ms < cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    for (int ch : {25, 50, 100}) {
        if (rc != LHMM_OK || ch == cur.graph_chunk) continue;
        lhmm_micro_config c = cur;
        c.graph_chunk = ch;
        double ms = 0.0;
        rc = trial(c, &ms);
        if (rc == LHMM_OK && ms < cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    if (rc != LHMM_OK) {
        (void)load();
        return done(rc);
    }
    rc = lhmm_micro_set_config(m, &cur);
    if (rc == LHMM_OK) {
        if (best) *best = cur;
        if (best_ms) *best_ms = cur_ms;
    }
    return done(rc);
}

int lhmm_micro_step_subset(lhmm_micro* m, const double* gradL, int32_t n_steps, double* stress_out,
                           const int32_t* boxes, int32_t n_sel) {
    g_err.clear();
    if (!m || !gradL || !stress_out) return fail(LHMM_ERR_ARG, "null argument");
    if (n_steps <= 0) return fail(LHMM_ERR_ARG, "n_steps must be positive (got %d)", n_steps);
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    const int bt = 256, bg = (m->n_boxes + bt - 1) / bt;
    HIPCHK(hipEventRecord(m->ev_in, m->user_stream));
    HIPCHK(hipStreamWaitEvent(m->stream, m->ev_in, 0));
    Ctx C{};
    int nblk = 0;
    int rc = select_boxes(m, boxes, n_sel, &C, &nblk);
    if (rc != LHMM_OK) return rc;
    k_setup_call<<<bg, bt, 0, m->stream>>>(m->ctx, gradL);
    k_zero_acc<<<(ACC * m->n_boxes + 255) / 256, 256, 0, m->stream>>>(m->ctx);
    launch_remove_mean(m, C, n_sel);
    if (!m->forces_valid) {
        launch_force_eval(m);
        m->forces_valid = true;
    }
    if (m->p.flags & LHMM_OPT_NO_GRAPH) {
        for (int k = 0; k < n_steps; ++k) launch_one_step_sel(m, C, n_sel, nblk);
    } else {
        const int chunk = n_steps < m->cfg.graph_chunk ? n_steps : m->cfg.graph_chunk;
        int done = 0;
        while (done < n_steps) {
            const int len = n_steps - done >= chunk ? chunk : n_steps - done;
            rc = launch_subset_steps(m, C, n_sel, nblk, len);
            if (rc != LHMM_OK) return rc;
            done += len;
        }
    }
    k_finalize<<<bg, bt, 0, m->stream>>>(m->ctx, stress_out, m->d_parts, 1.0 / n_steps);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(m->ev_out, m->stream));
    HIPCHK(hipStreamWaitEvent(m->user_stream, m->ev_out, 0));
    return LHMM_OK;
}

int lhmm_micro_snapshot(lhmm_micro* m) {
    g_err.clear();
    if (!m) return fail(LHMM_ERR_ARG, "null argument");
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    const size_t bytes = 3 * (size_t)m->n_total * m->real_size;
    if (!m->d_snap_s) {
        int rc = dalloc((char**)&m->d_snap_s, bytes);
        if (rc == LHMM_OK) rc = dalloc((char**)&m->d_snap_c, bytes);
        if (rc == LHMM_OK) rc = dalloc((char**)&m->d_snap_f, bytes);
        if (rc == LHMM_OK) rc = dalloc(&m->d_snap_dyn, m->n_boxes);
        if (rc != LHMM_OK) return rc;
    }
    HIPCHK(hipEventRecord(m->ev_in, m->user_stream));
    HIPCHK(hipStreamWaitEvent(m->stream, m->ev_in, 0));
    if (!m->forces_valid) {
        launch_force_eval(m);
        m->forces_valid = true;
    }
    HIPCHK(hipMemcpyAsync(m->d_snap_s, m->d_s, bytes, hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->d_snap_c, m->d_c, bytes, hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->d_snap_f, m->d_f, bytes, hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->d_snap_dyn, m->d_dyn, sizeof(BoxDyn) * m->n_boxes, hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipEventRecord(m->ev_out, m->stream));
    HIPCHK(hipStreamWaitEvent(m->user_stream, m->ev_out, 0));
    m->have_snapshot = true;
    return LHMM_OK;
}

int lhmm_micro_restore(lhmm_micro* m, const int32_t* boxes, int32_t n_sel) {
    g_err.clear();
    if (!m) return fail(LHMM_ERR_ARG, "null argument");
    if (!m->have_snapshot) return fail(LHMM_ERR_STATE, "no snapshot taken");
    HIPCHK(hipEventRecord(m->ev_in, m->user_stream));
    HIPCHK(hipStreamWaitEvent(m->stream, m->ev_in, 0));
    Ctx C{};
    int nblk = 0;
    int rc = select_boxes(m, boxes, n_sel, &C, &nblk);
    if (rc != LHMM_OK) return rc;
    if (m->precision == LHMM_FP64)
        k_restore<double><<<n_sel, 256, 0, m->stream>>>(C, (const double*)m->d_snap_s, (const double*)m->d_snap_c,
                                                        (const double*)m->d_snap_f, m->d_snap_dyn);
    else
        k_restore<float><<<n_sel, 256, 0, m->stream>>>(C, (const float*)m->d_snap_s, (const float*)m->d_snap_c,
                                                       (const float*)m->d_snap_f, m->d_snap_dyn);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(m->ev_out, m->stream));
    HIPCHK(hipStreamWaitEvent(m->user_stream, m->ev_out, 0));
    return LHMM_OK;
}

int lhmm_micro_forces(lhmm_micro* m, const double* gradL, double* f_out, double* virial_out) {
    g_err.clear();
    if (!m || !gradL || !f_out) return fail(LHMM_ERR_ARG, "null argument");
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    for (int k = 0; k < 9 * m->n_boxes; ++k)
        if (!std::isfinite(gradL[k])) return fail(LHMM_ERR_ARG, "gradient not finite");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    HIPCHK(hipMemcpy(m->d_gradL, gradL, 9 * m->n_boxes * sizeof(double), hipMemcpyHostToDevice));
    const int bt = 256, bg = (m->n_boxes + bt - 1) / bt;
    k_setup_call<<<bg, bt, 0, m->stream>>>(m->ctx, m->d_gradL);
    launch_force_eval(m);
    HIPCHK(hipGetLastError());
    rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    m->forces_valid = false;  // the next step recomputes forces with its own gradient
    const size_t N = (size_t)m->n_total;
    std::vector<char> buf(3 * N * m->real_size + 1);
    HIPCHK(hipMemcpy(buf.data(), m->d_f, 3 * N * m->real_size, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < N; ++i)
        for (int k = 0; k < 3; ++k)
            f_out[3 * i + k] = m->precision == LHMM_FP64 ? ((double*)buf.data())[k * N + i]
                                                         : (double)((float*)buf.data())[k * N + i];
    if (virial_out) {
        const size_t ps = (size_t)m->ctx.pv_stride;
        std::vector<double> pv((size_t)m->n_blocks * ps);
        HIPCHK(hipMemcpy(pv.data(), m->d_part_vir, pv.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int b = 0; b < m->n_boxes; ++b) {
            double* o = virial_out + 12 * b;
            for (int q = 0; q < 12; ++q) o[q] = 0.0;
            for (int k = 0; k < m->box[b].nblk; ++k)
                for (int q = 0; q < 12; ++q) o[q] += pv[ps * (size_t)(m->box[b].blk_off + k) + q];
            for (int q = 0; q < 6; ++q) o[q] *= m->ctx.vir_scale;  // ordered pairs count each pair twice
        }
    }
    return LHMM_OK;
}

int lhmm_micro_time(lhmm_micro* m, const double* gradL, int32_t n_steps, double* avg_ms, double* stress_out) {
    g_err.clear();
    if (!m || !gradL || !avg_ms) return fail(LHMM_ERR_ARG, "null argument");
    if (n_steps <= 0) return fail(LHMM_ERR_ARG, "n_steps must be positive (got %d)", n_steps);
    if (!m->have_state) return fail(LHMM_ERR_STATE, "no particle state loaded");
    const int bt = 256, bg = (m->n_boxes + bt - 1) / bt;
    hipEvent_t ev[2 * LHMM_N_KERNELS];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(m->ev_in, m->user_stream));
    HIPCHK(hipStreamWaitEvent(m->stream, m->ev_in, 0));
    k_setup_call<<<bg, bt, 0, m->stream>>>(m->ctx, gradL);
    k_zero_acc<<<(ACC * m->n_boxes + 255) / 256, 256, 0, m->stream>>>(m->ctx);
    launch_remove_mean(m, m->ctx, m->n_boxes);
    if (!m->forces_valid) {
        launch_force_eval(m);
        m->forces_valid = true;
    }
    double sum[LHMM_N_KERNELS] = {0, 0, 0, 0, 0, 0};
    int rc = LHMM_OK;
    for (int k = 0; k < n_steps && rc == LHMM_OK; ++k) {
        if (m->precision == LHMM_FP64)
            launch_step_timed<double>(m, ev);
        else
            launch_step_timed<float>(m, ev);
        hipError_t e = hipEventSynchronize(ev[2 * LHMM_N_KERNELS - 1]);
        if (e != hipSuccess) {
            rc = fail(LHMM_ERR_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
            break;
        }
        for (int q = 0; q < LHMM_N_KERNELS; ++q) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]) != hipSuccess) {
                rc = fail(LHMM_ERR_HIP, "hipEventElapsedTime failed");
                break;
            }
            sum[q] += ms;
        }
    }
    if (rc == LHMM_OK) {
        for (int q = 0; q < LHMM_N_KERNELS; ++q) avg_ms[q] = sum[q] / n_steps;
        if (stress_out) k_finalize<<<bg, bt, 0, m->stream>>>(m->ctx, stress_out, m->d_parts, 1.0 / n_steps);
        hipError_t e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) rc = fail(LHMM_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
}

int lhmm_micro_stress_parts(lhmm_micro* m, double* parts_out) {
    g_err.clear();
    if (!m || !parts_out) return fail(LHMM_ERR_ARG, "null argument");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    std::vector<double> v((size_t)ACC * m->n_boxes);
    HIPCHK(hipMemcpy(v.data(), m->d_parts, v.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int b = 0; b < m->n_boxes; ++b)
        for (int q = 0; q < 18; ++q) parts_out[18 * (size_t)b + q] = v[(size_t)ACC * b + q];
    return LHMM_OK;
}

int lhmm_micro_components(lhmm_micro* m, double* out) {
    g_err.clear();
    if (!m || !out) return fail(LHMM_ERR_ARG, "null argument");
    if (!(m->p.flags & LHMM_OPT_COMPONENTS))
        return fail(LHMM_ERR_STATE, "the engine was created without LHMM_OPT_COMPONENTS");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    std::vector<double> v((size_t)ACC * m->n_boxes);
    HIPCHK(hipMemcpy(v.data(), m->d_parts, v.size() * sizeof(double), hipMemcpyDeviceToHost));
    // sums: kinetic 0, pair 6, FENE 12, C 18, D 24, R 30 -> kin, C, D, R, FENE
    const int src[5] = {0, 18, 24, 30, 12};
    for (int b = 0; b < m->n_boxes; ++b)
        for (int part = 0; part < 5; ++part)
            for (int q = 0; q < 6; ++q) out[30 * (size_t)b + 6 * part + q] = v[(size_t)ACC * b + src[part] + q];
    return LHMM_OK;
}

int lhmm_micro_pair_total(lhmm_micro* m, uint64_t* pairs_out) {
    g_err.clear();
    if (!m || !pairs_out) return fail(LHMM_ERR_ARG, "null argument");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    std::vector<unsigned long long> v(m->n_boxes);
    HIPCHK(hipMemcpy(v.data(), m->d_tot_pairs, m->n_boxes * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int b = 0; b < m->n_boxes; ++b) pairs_out[b] = v[b];
    return LHMM_OK;
}

int lhmm_micro_prepare(lhmm_micro* m, int32_t n_steps) {
    g_err.clear();
    if (!m) return fail(LHMM_ERR_ARG, "null engine");
    if (n_steps <= 0) return fail(LHMM_ERR_ARG, "n_steps must be positive (got %d)", n_steps);
    if (m->p.flags & LHMM_OPT_NO_GRAPH) return LHMM_OK;
    const int chunk = n_steps < m->cfg.graph_chunk ? n_steps : m->cfg.graph_chunk;
    hipGraphExec_t g = nullptr;
    int rc = get_graph(m, chunk, &g);
    if (rc == LHMM_OK && n_steps % chunk) rc = get_graph(m, n_steps % chunk, &g);
    return rc;
}

int lhmm_micro_pair_counts(lhmm_micro* m, uint64_t* pairs_out) {
    g_err.clear();
    if (!m || !pairs_out) return fail(LHMM_ERR_ARG, "null argument");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    std::vector<unsigned long long> v(m->n_boxes);
    HIPCHK(hipMemcpy(v.data(), m->d_acc_pairs, m->n_boxes * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int b = 0; b < m->n_boxes; ++b) pairs_out[b] = v[b];
    return LHMM_OK;
}

int lhmm_micro_flags(lhmm_micro* m, uint32_t* flags_out, int32_t clear) {
    g_err.clear();
    if (!m || !flags_out) return fail(LHMM_ERR_ARG, "null argument");
    int rc = sync_engine(m);
    if (rc != LHMM_OK) return rc;
    HIPCHK(hipMemcpy(flags_out, m->d_flags, m->n_boxes * sizeof(unsigned), hipMemcpyDeviceToHost));
    if (clear) HIPCHK(hipMemset(m->d_flags, 0, m->n_boxes * sizeof(unsigned)));
    return LHMM_OK;
}

int lhmm_micro_sizes(const lhmm_micro* m, int64_t* n_total, int32_t* n_boxes) {
    g_err.clear();
    if (!m) return fail(LHMM_ERR_ARG, "null engine");
    if (n_total) *n_total = m->n_total;
    if (n_boxes) *n_boxes = m->n_boxes;
    return LHMM_OK;
}

int lhmm_micro_destroy(lhmm_micro* m) {
    g_err.clear();
    if (!m) return LHMM_OK;
    release(m);
    delete m;
    return LHMM_OK;
}

}  // extern "C"
