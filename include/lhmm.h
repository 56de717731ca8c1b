/*
 * lhmm.h -- C ABI of the MI355X (gfx950) micro-DPD engine of the Lagrangian
 * Heterogeneous Multiscale Method (LHMM, DPD-SPH).
 *
 * The engine advances many independent periodic micro-boxes, one per SPH
 * macro particle.  Each box holds DPD solvent and FENE bead-spring chains;
 * each is driven by its particle's velocity gradient and returns the
 * Irving-Kirkwood stress averaged over the exchange interval:
 *   - pair forces: conservative, dissipative and random forces of the
 *     micro-scale model (paper Sec. "Microscale: Polymer Melt Model -- DPD
 *     and FENE", Eqs. F_DPD, conservative, dissipative, random) with
 *     w^D = (w^R)^2, w^R = 1 - r/rc, sigma^2 = 2 gamma kBT and the discrete
 *     random force scaled by 1/sqrt(dt);
 *   - bonds: attractive FENE springs (Eq. fene_force);
 *   - integration: velocity-Verlet of Eq. (motion) (Appendix "Detailed
 *     Coupling Protocol", Step 3) in a periodic cell deformed by the imposed
 *     gradient, dh/dt = L h, with peculiar velocities c = v - L r;
 *   - imposed flow: the macro-to-micro coupling of Eq. (micro_bc), v = L r,
 *     applied homogeneously through the deforming cell (Lees-Edwards for
 *     simple shear);
 *   - stress: Eqs. (IKtotal), (kinetic_stress), (potential_stress); with a
 *     uniform weight over the periodic cell the Irving-Kirkwood stress is the
 *     virial stress  sigma = -(sum m c (x) c + sum_pairs d (x) f) / V,
 *     tension positive, averaged over the steps of the exchange interval
 *     (Sec. "Micro-to-macro Coupling");
 *   - micro boxes persist between calls (continuous-intermittent coupling,
 *     Sec. "Temporal Coupling Scheme").
 *
 * Results are reproducible bit for bit: every sum has a fixed order (no
 * floating-point atomics to global memory).
 *
 * Conventions
 *   - Matrices are 3x3 row-major doubles.  A cell h has the lattice vectors
 *     as columns (r = h s, s in [0,1)^3).  A velocity gradient L maps
 *     position to streaming velocity, u = L r; it must be in-plane (zero
 *     z row and column) and traceless.  Simple shear u_x = g y is L[1] = g.
 *   - Stress vectors are (xx, yy, zz, xy, xz, yz).
 *   - Particles of all boxes are concatenated in box order; inside a box,
 *     particle k has id k; ids 0 .. n_chains*chain_len-1 form chains of
 *     chain_len consecutive ids, the rest are solvent.
 *   - Every function returns LHMM_OK (0) or a negative LHMM_ERR_* code and
 *     never aborts; lhmm_last_error() returns a thread-local message.
 *   - Per-box physics flags (LHMM_FLAG_*) are sticky and are read with
 *     lhmm_micro_flags; a flagged box does not stop the batch.
 *   - The engine owns all device memory it allocates.  Pointer arguments
 *     are borrowed for the duration of the call.  Which arguments are host
 *     and which are device pointers is stated per function.
 *   - Device work runs on a stream the engine creates (default priority).
 *     Calls taking device pointers are ordered after prior work on the
 *     caller's stream and make the caller's stream wait for their results.
 */
#ifndef LHMM_H
#define LHMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LHMM_OK 0
#define LHMM_ERR_ARG (-1)   /* invalid argument (shape, range, NaN, null)   */
#define LHMM_ERR_HIP (-2)   /* a HIP runtime call failed                     */
#define LHMM_ERR_OOM (-3)   /* device or host allocation failed              */
#define LHMM_ERR_STATE (-4) /* call out of order (e.g. step before state)    */

#define LHMM_FLAG_BOND 1u      /* a bond reached r >= R0 (force clamped)    */
#define LHMM_FLAG_CELL 2u      /* a cell width fell below 3 rc              */
#define LHMM_FLAG_NONFINITE 4u /* a stress sample was not finite            */
#define LHMM_FLAG_ARG 8u       /* the box's gradient was rejected (L := 0)  */
/* the reduced cell's smallest width fell below LHMM_THIN_WIDTH rc: the box
 * is still exact, but a flow that keeps stretching it will reach the
 * LHMM_FLAG_CELL guard; long runs under time-varying gradients restore or
 * re-initialise such boxes */
#define LHMM_FLAG_THIN 16u
#define LHMM_THIN_WIDTH 3.3

#define LHMM_FP32 0 /* single-precision particle state and pair forces     */
#define LHMM_FP64 1 /* double-precision particle state and pair forces     */

#define LHMM_OPT_NO_GRAPH 1 /* launch every kernel eagerly (no HIP graphs) */
/* keep the virials of the conservative, dissipative and random pair forces
 * apart (lhmm_micro_components); the steps use a variant of the pair-force
 * kernel with 18 more accumulators, and the pair stress they return is
 * summed exactly as without the option */
#define LHMM_OPT_COMPONENTS 2

typedef struct lhmm_micro lhmm_micro;

/* Model parameters, shared by every box (reduced units m = rc = kBT = 1 in
 * the paper's Table "DPD and FENE simulation parameters"). */
typedef struct {
    double a;        /* conservative amplitude a_ij                          */
    double gamma;    /* dissipative amplitude gamma^D                        */
    double sigma;    /* random amplitude sigma^R (= sqrt(2 gamma kBT))       */
    double kBT;      /* thermal energy                                       */
    double mass;     /* bead mass                                            */
    double rc;       /* cutoff radius                                        */
    double dt;       /* micro time step                                      */
    double H;        /* FENE spring constant                                 */
    double R0;       /* FENE maximum extension                               */
    uint64_t seed;   /* key of the counter-based random stream               */
    int32_t chain_len;  /* beads per chain N_d (>= 2)                        */
    int32_t precision;  /* LHMM_FP32 or LHMM_FP64                            */
    int32_t flags;      /* LHMM_OPT_* bits                                   */
} lhmm_params;

/* One micro-box. */
typedef struct {
    int32_t n_particles; /* >= 2                                             */
    int32_t n_chains;    /* n_chains * chain_len <= n_particles              */
    uint32_t rng_id;     /* box word of the random-force counter, usually the */
                         /* SPH particle index; equal ids draw equal noise    */
    int32_t reserved;    /* must be 0                                         */
    double h0[9];        /* initial cell; in-plane basis in columns 0-1, z   */
                         /* extent h0[8] > 0, zero z coupling, det > 0        */
} lhmm_box;

/* Initial cell of a box that must stay usable under a constant in-plane
 * gradient (host computation only, no device work; reentrant).  The
 * homogeneous imposition of the macro gradient (Eq. micro_bc) deforms the
 * periodic cell as dh/dt = L h; the returned cell keeps its reduced
 * lattice's perpendicular widths large for the run:
 *   LHMM_CELL_CUBIC:   the cube of side edge, kept when its reduced lattice
 *                      stays at least min_width wide over [0, t_run];
 *   LHMM_CELL_ROTATED: otherwise, for a rotational or shear-like gradient
 *                      (a^2 + bc <= 0, L = [[a, b], [c, -a]] in the plane),
 *                      the square of side edge rotated (46 angles of
 *                      [0, pi/2)) to the angle whose narrowest width over
 *                      [0, t_run] is largest;
 *   LHMM_CELL_KR:      otherwise (hyperbolic gradient, k^2 = a^2 + bc > 0), a
 *                      lattice aligned in the manner of Kraynik and Reinelt:
 *                      exp(L T) P = P M with M = [[2, 1], [1, 1]] and
 *                      T = ln((3 + sqrt 5)/2) / k, so the flow maps it onto
 *                      itself every period; among the family
 *                      V diag(r, +-1) W^-1 (V, W eigenvectors of L and M,
 *                      r = e^-4 .. e^4 in 81 steps) of area edge^2, the
 *                      member whose narrowest width over a period is
 *                      largest; the members are time shifts of one
 *                      lattice, so among those within 1e-9 of the best the
 *                      one widest at t = 0 is taken.
 * L: host 9 doubles (u = L r; in-plane and traceless); h_out: host 9
 * doubles, the in-plane basis reduced (its two successive minima, det > 0)
 * and z extent edge; kind: host, may be NULL.  Errors: ARG (bad L, edge,
 * t_run or min_width). */
#define LHMM_CELL_CUBIC 0
#define LHMM_CELL_KR 1
#define LHMM_CELL_ROTATED 2
int lhmm_box_cell(const double* L, double edge, double t_run, double min_width, double* h_out, int32_t* kind);

/* Allocate an engine for n_boxes boxes.  p, boxes: host.  stream: the
 * caller's hipStream_t (may be NULL for the null stream).  The particle
 * state is undefined until lhmm_micro_set_state.  Errors: ARG, HIP, OOM. */
int lhmm_micro_create(const lhmm_params* p, const lhmm_box* boxes, int32_t n_boxes, void* stream,
                      lhmm_micro** out);

/* Load the particle state of every box.  s, c: host, n_total x 3 doubles
 * (row per particle, boxes concatenated): fractional coordinates in [0,1)
 * and peculiar velocities.  f: host n_total x 3, the forces the next step
 * starts from (as returned by lhmm_micro_get_state, for an exact resume),
 * or NULL to recompute them at the next step call with that call's
 * gradient.  h: host, n_boxes x 9, current cells (NULL keeps the cells).
 * step: completed steps (the random-force counter).  Values are rounded to
 * the engine's precision.  Synchronous.  Errors: ARG (NaN, s outside [0,1),
 * bad cell). */
int lhmm_micro_set_state(lhmm_micro* m, const double* s, const double* c, const double* f, const double* h,
                         uint64_t step);

/* Read the particle state back.  s, c, f: host n_total x 3 (f: the forces
 * carried into the next step); h: host n_boxes x 9; step: host.  Any of
 * them may be NULL.  Synchronous. */
int lhmm_micro_get_state(lhmm_micro* m, double* s, double* c, double* f, double* h, uint64_t* step);

/* Advance every box by n_steps velocity-Verlet steps under its own constant
 * gradient and write the mean stress over those steps.
 *   gradL: DEVICE pointer, n_boxes x 9 doubles (u = L r per box);
 *   stress_out: DEVICE pointer, n_boxes x 6 doubles.
 * A gradient that is not finite, in-plane and traceless sets LHMM_FLAG_ARG
 * on its box, which then advances with L = 0.  Every call (and every call of
 * lhmm_micro_step_subset and lhmm_micro_time, for the boxes it advances)
 * first removes each box's mean peculiar velocity: the micro-domain moves
 * with its macro particle, and since pair forces cancel, the mean would
 * otherwise follow d<c>/dt = -L <c> and grow wherever the flow compresses
 * the box, seeded by rounding.  Asynchronous with respect to the host;
 * ordered on the caller's stream.  Errors: ARG (n_steps <= 0), STATE (no
 * state loaded), HIP. */
int lhmm_micro_step(lhmm_micro* m, const double* gradL, int32_t n_steps, double* stress_out);

/* As lhmm_micro_step, for the listed boxes only: boxes is a HOST array of
 * n_sel strictly increasing box indices; the launches cover just their
 * particles and cells.  The other boxes keep their state; their rows of
 * stress_out are written as zero.  Every step advances the shared random-
 * force counter once, so a selected box follows exactly the trajectory a
 * full lhmm_micro_step would give it from the same state and counter.
 * Used where only some micro-domains must run (the surrogate's fallback
 * boxes).  Waits for the upload of the previous call's list.  Errors: ARG
 * (empty, unsorted or out-of-range list), STATE, HIP. */
int lhmm_micro_step_subset(lhmm_micro* m, const double* gradL, int32_t n_steps, double* stress_out,
                           const int32_t* boxes, int32_t n_sel);

/* Launch parameters of the step kernels.  None of them changes a result:
 * every sum keeps its order, so all configurations give bit-identical
 * trajectories.
 *   queue_depth: per-lane neighbour queue of the pair-force kernel
 *                (2, 4, 8, 16, 32 entries of 4 bytes);
 *   drain:       evaluation rounds run until every queue holds at most this
 *                many neighbours (0 .. queue_depth - u, where a search
 *                iteration tests u = 4, 2, 1 records per lane for depths
 *                >= 8, 4, 2 before the queues are checked again);
 *   busy_lanes:  the search also stops, and rounds also continue, while at
 *                least this many of a wave's 64 lanes hold a neighbour
 *                (1 .. 64; 65 turns the rule off);
 *   bin_threads: threads of the per-box binning workgroup (256, 512, 1024);
 *   graph_chunk: micro steps per captured HIP graph (1 .. 1000);
 *   prune:       1 skips stencil cells that lie provably beyond the cutoff
 *                (the accepted pairs and their order are unchanged), 0
 *                scans the full 27-cell stencil;
 *   fuse_bin:    1 runs the cell step and the half kick and drift inside the
 *                per-box binning workgroup (two launches fewer per step;
 *                lhmm_micro_time then reports their time under binning);
 *   groups:      1 .. 4: with fused binning, a captured step splits the
 *                boxes by particle count into this many groups (the largest
 *                boxes, two thirds of the particles, in the last), each
 *                binned and force-evaluated on its own stream, so that the
 *                force pass of small boxes runs while large boxes are still
 *                being binned (1: one stream);
 *   bin_split:   0, or 256 .. 4096: with groups > 1 the group of the largest
 *                boxes is binned by several workgroups per box, over chunks
 *                of this many particles (count, scan and scatter passes), so
 *                that one box's sort is not held by one compute unit. */
typedef struct {
    int32_t queue_depth;
    int32_t drain;
    int32_t busy_lanes;
    int32_t bin_threads;
    int32_t graph_chunk;
    int32_t prune;
    int32_t fuse_bin;
    int32_t groups;
    int32_t bin_split;
} lhmm_micro_config;

/* Set / read the launch parameters (defaults: depth 16, drain 12; busy rule
 * off; 1024 binning threads; fused binning; two box groups; no split
 * binning (measured slower); 50-step graphs; no pruning: with
 * cells barely wider than the cutoff it skips little and costs more).  Set waits for the
 * engine and drops its captured graphs.  Errors: ARG. */
int lhmm_micro_set_config(lhmm_micro* m, const lhmm_micro_config* cfg);
int lhmm_micro_get_config(lhmm_micro* m, lhmm_micro_config* cfg);

/* Choose the launch parameters for the loaded boxes by timing: a coordinate
 * search over (queue_depth, drain, busy_lanes), then bin_threads, fuse_bin, prune, groups, graph_chunk,
 * each candidate timed over trial_steps steps (after trial_steps warm-up
 * steps) under gradL (DEVICE n_boxes x 9) with HIP events.  The particle
 * state, cells, flags and random-force counter are put back after every
 * trial, so tuning does not change the trajectory.  The best configuration
 * is set and returned in best (HOST, may be NULL) with its time per step in
 * best_ms (HOST, may be NULL).  Synchronous; allocates a temporary copy of
 * the state.  Errors: ARG, STATE, OOM, HIP. */
int lhmm_micro_autotune(lhmm_micro* m, const double* gradL, int32_t trial_steps, lhmm_micro_config* best,
                        double* best_ms);

/* Turn listed boxes into micro-domains with boundary regions (Sec.
 * "Macro-to-Micro Coupling", Tab. 2: core, boundary-condition region,
 * buffer).  regions: HOST n_boxes x 2 doubles (hc, hb) per box; (0, 0)
 * leaves a box as it is.  For a box with 0 < hc <= hb, a particle's in-plane
 * position r' relative to the cell's centre puts it in the core
 * (max(|x'|, |y'|) < hc), the boundary-condition ring (hc <= .. < hb) or the
 * buffer (beyond); hb may not exceed half the cell's in-plane width.  Such a
 * box's cell no longer deforms: the gradient of each later step call is the
 * imposed field G of Eq. (micro_bc), v' = G r', toward which the ring's
 * in-plane velocities relax after each half kick,
 *   c <- u + (c - u) exp(-zeta dt/2) + sqrt(kBT/m (1 - exp(-zeta dt))) xi,
 * u = G r' (an exact Ornstein-Uhlenbeck step; xi a normal pair of the
 * random stream at counter (id, 0xFFFFFFF0 + half kick, step, box)); the
 * core and the buffer move freely (the buffer is the reservoir between the
 * ring and its periodic images).  Its stress is the Irving-Kirkwood stress
 * of the core (Eqs. IKtotal, kinetic_stress, potential_stress with a weight
 * uniform over the core): the kinetic part over the core's particles with
 * their velocity relative to G r', each pair's and bond's d (x) f weighted by
 * the fraction of its segment inside the core, over the core's volume
 * (2 hc)^2 h_zz.  zeta >= 0 is shared by the engine's boxes.  Synchronous;
 * drops captured graphs.  Errors: ARG, HIP. */
int lhmm_micro_set_afbc(lhmm_micro* m, const double* regions, double zeta);

/* Keep a device copy of the current state of every box (positions,
 * velocities, forces, cell).  Ordered on the caller's stream.  Errors:
 * STATE (no state loaded), OOM, HIP. */
int lhmm_micro_snapshot(lhmm_micro* m);

/* Return the listed boxes (HOST, strictly increasing) to their snapshot
 * state and clear their flags; the random-force counter is not rewound.
 * Ordered on the caller's stream.  Errors: ARG, STATE (no snapshot), HIP. */
int lhmm_micro_restore(lhmm_micro* m, const int32_t* boxes, int32_t n_sel);

/* Forces at the current state with random-force counter = current step,
 * without advancing: f_out host n_total x 3; virial_out host n_boxes x 12
 * (sum over pairs of d (x) f for the DPD pairs, then for the FENE bonds,
 * each xx,yy,zz,xy,xz,yz; may be NULL).  gradL: host n_boxes x 9.
 * Synchronous.  Errors: ARG, STATE, HIP. */
int lhmm_micro_forces(lhmm_micro* m, const double* gradL, double* f_out, double* virial_out);

/* Mean stress parts of the last lhmm_micro_step call: host n_boxes x 3 x 6
 * (kinetic, DPD pairs, FENE bonds; their sum is the stress).  Synchronous. */
int lhmm_micro_stress_parts(lhmm_micro* m, double* parts_out);

/* Mean stress of the last lhmm_micro_step call by force type, Eqs.
 * (IKtotal), (kinetic_stress), (potential_stress): host n_boxes x 5 x 6 in
 * the order kinetic, conservative (Eq. conservative), dissipative (Eq.
 * dissipative), random (Eq. random), FENE (Eq. fene_force); their sum is the
 * stress.  Needs LHMM_OPT_COMPONENTS at create (else STATE).  Synchronous. */
int lhmm_micro_components(lhmm_micro* m, double* out);

/* Unordered DPD pairs within the cutoff, summed over the steps of the last
 * lhmm_micro_step call: host n_boxes uint64.  Synchronous. */
int lhmm_micro_pair_counts(lhmm_micro* m, uint64_t* pairs_out);

/* The same count summed over every step of every call (full, subset and
 * timed steps, fallback replays included) since the engine was created:
 * host n_boxes uint64.  Synchronous. */
int lhmm_micro_pair_total(lhmm_micro* m, uint64_t* pairs_out);

/* Capture and instantiate the HIP graphs a later lhmm_micro_step call of
 * n_steps steps will replay (a graph of graph_chunk steps and one of the
 * remainder), without running any step, so that the first such call does
 * no capture.  No effect with LHMM_OPT_NO_GRAPH.  Errors: ARG, HIP. */
int lhmm_micro_prepare(lhmm_micro* m, int32_t n_steps);

/* Sticky physics flags per box: host n_boxes uint32 (LHMM_FLAG_*).
 * clear != 0 resets them after reading.  Synchronous. */
int lhmm_micro_flags(lhmm_micro* m, uint32_t* flags_out, int32_t clear);

/* Kernels of one micro step, in launch order (indices of lhmm_micro_time). */
#define LHMM_K_CELL 0       /* cell deformation, reduction, grid (per box)   */
#define LHMM_K_KICK_DRIFT 1 /* half kick, drift, wrap, cell index            */
#define LHMM_K_BIN 2        /* counting sort by cell (per box)               */
#define LHMM_K_FORCES 3     /* DPD pair forces, FENE bonds, virial           */
#define LHMM_K_KICK2 4      /* second half kick (inside the force kernel: 0) */
#define LHMM_K_STRESS 5     /* per-box stress of the step, accumulation      */
#define LHMM_N_KERNELS 6

/* Advance like lhmm_micro_step (same kernels, grids and state update) but
 * launch eagerly with a HIP event pair around every kernel on the engine's
 * stream, and return each kernel's mean duration in milliseconds.
 *   gradL: DEVICE pointer n_boxes x 9; avg_ms: host LHMM_N_KERNELS doubles;
 *   stress_out: DEVICE pointer n_boxes x 6 (may be NULL).
 * Synchronous.  Errors: ARG, STATE, HIP. */
int lhmm_micro_time(lhmm_micro* m, const double* gradL, int32_t n_steps, double* avg_ms, double* stress_out);

/* Sizes: total particles and boxes.  Host pointers, may be NULL. */
int lhmm_micro_sizes(const lhmm_micro* m, int64_t* n_total, int32_t* n_boxes);

/* Release every resource of the engine (waits for its stream).  NULL ok. */
int lhmm_micro_destroy(lhmm_micro* m);

/* ------------------------------------------------------------------------
 * Macro side: 2-D SPH in a periodic box and the coupled exchange interval.
 *   - number density d_I = sum_J W(r_IJ), rho_I = m d_I, Tait pressure
 *     p = c^2 rho0/7 ((rho/rho0)^7 - 1) + theta c^2 rho0/7 (Eq. tait);
 *   - momentum, Eq. (sph_continuity): pressure, viscous (a = 2 eta - zeta,
 *     b = 4 zeta + 2 eta) and micro-to-macro polymer terms, plus a body
 *     force per unit mass (force_mode: reversing at mid-height for the
 *     reverse Poiseuille flow, or uniform);
 *   - obstacles: the last n_fixed particles are frozen wall particles (the
 *     paper does not say how its cylinders are represented).  They enter
 *     every sum as neighbours (density, pressure from their own density,
 *     the viscous term with their velocity) but never move, carry no
 *     micro-domain and no polymer stress (their rows of sigma are ignored),
 *     and get zero gradient rows;
 *   - kernel of support radius h (kernel): the quintic spline
 *     W = 63/(478 pi h^2) [(3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5]_+, q = 3 r / h,
 *     or the 2-D Lucy kernel of Appendix "Kernel function approximation",
 *     Eq. (lucy_kernel), W = 5/(pi h^2) (1 + 3q)(1 - q)^3, q = r / h < 1
 *     (the paper's choice, with h = 4 dh);
 *   - velocity-Verlet steps (Appendix "Detailed Coupling Protocol");
 *   - velocity gradient for the micro-domains, Eq. (macro_micro) with the
 *     volume factor 1/d_J; the micro-domain of particle I is driven by
 *     L_I = lambda* x the traceless part of (grad v_I)^T (the isochoric part
 *     of the weakly compressible flow);
 *   - the polymer stress fed back is alpha/lambda* x the in-plane part of
 *     the micro-domain's deviatoric mean stress (Eq. pip): an isotropic micro
 *     stress (3-D boxes) or an isotropic in-plane stress (planar cells, see
 *     micro_dim) feeds back nothing; the macro EOS supplies the pressure.
 * ------------------------------------------------------------------------ */
typedef struct lhmm_sph lhmm_sph;

typedef struct {
    double rho0;        /* reference density                                 */
    double eta;         /* solvent shear viscosity eta_s                     */
    double zeta;        /* solvent bulk viscosity                            */
    double c;           /* artificial sound speed                            */
    double theta;       /* background-pressure factor (< 1)                  */
    double F;           /* body force magnitude per unit mass                */
    double h;           /* kernel support radius                             */
    double dt;          /* macro time step                                   */
    double mass;        /* particle mass                                     */
    double Lx, Ly;      /* periodic box                                      */
    double lambda_star; /* time-scale ratio lambda*                          */
    double alpha;       /* viscosity ratio alpha                             */
    int32_t n_fixed;    /* trailing wall particles (see below)               */
    int32_t force_mode; /* LHMM_FORCE_REVERSE or LHMM_FORCE_UNIFORM          */
    int32_t kernel;     /* LHMM_KERNEL_QUINTIC or LHMM_KERNEL_LUCY           */
    int32_t micro_dim;  /* dimension of the micro-domains: 3 (or 0) for 3-D  */
                        /* boxes, whose deviatoric part removes tr/3; 2 for  */
                        /* planar cells (no zz stress), whose in-plane       */
                        /* deviatoric part removes (xx + yy)/2               */
} lhmm_sph_params;

#define LHMM_FORCE_REVERSE 0 /* +F x-hat where y >= Ly/2, -F below            */
#define LHMM_FORCE_UNIFORM 1 /* +F x-hat everywhere                          */
#define LHMM_KERNEL_QUINTIC 0 /* quintic spline, support h                   */
#define LHMM_KERNEL_LUCY 1    /* Lucy kernel, Eq. (lucy_kernel), support h   */

/* Allocate an SPH engine of n particles.  r0, v0: host n x 2.  stream: the
 * caller's hipStream_t (all SPH work is launched on it).  Errors: ARG, HIP,
 * OOM. */
int lhmm_sph_create(const lhmm_sph_params* p, int32_t n, const double* r0, const double* v0, void* stream,
                    lhmm_sph** out);

/* One velocity-Verlet step with the polymer stress of the given micro
 * stresses held fixed, then the micro-domain gradients at the new state.
 *   sigma: DEVICE n x 6 (micro mean stresses xx,yy,zz,xy,xz,yz) or NULL for
 *          no polymer stress;
 *   gradL_out: DEVICE n x 9 (may be NULL).
 * Asynchronous on the engine's stream.  Errors: ARG, HIP. */
int lhmm_sph_step(lhmm_sph* s, const double* sigma, double* gradL_out);

/* State to host: r, v n x 2, d n (any may be NULL).  Synchronous. */
int lhmm_sph_get_state(lhmm_sph* s, double* r, double* v, double* d);

/* Host copies of the coupling state kept by the engine for
 * lhmm_couple_step: the micro stresses of the last interval (n x 6) and the
 * micro gradients of the last SPH step (n x 9); either may be NULL.
 * Synchronous. */
int lhmm_sph_coupling_state(lhmm_sph* s, double* sigma, double* gradL);

/* One exchange interval delta_t = m_bar dt_SPH = k_micro dt_micro of the
 * coupling protocol (Appendix "Detailed Coupling Protocol", Steps 1-4;
 * Sec. "Temporal Coupling Scheme"): m_bar SPH steps with the stored micro
 * stresses held fixed, the velocity gradients at the end of the last one to
 * the micro-domains, k_micro micro steps of every box, their mean stresses
 * stored for the next interval.  The micro engine must hold one box per
 * mobile SPH particle, in order, and both engines must have been created on
 * the same stream.  m_bar, k_micro >= 1.  No host synchronisation.
 * Errors: ARG, STATE, HIP. */
int lhmm_couple_step(lhmm_sph* s, lhmm_micro* m, int32_t m_bar, int32_t k_micro);

int lhmm_sph_destroy(lhmm_sph* s);

/* ------------------------------------------------------------------------
 * Stress surrogate: an ensemble of n_members independent MLPs
 *   x -> GELU(x W1 + b1) -> GELU(. W2 + b2) -> . W3 + b3
 * (GELU in the erf form) mapping a particle's recent history of micro
 * velocity gradients to the deviatoric micro stress, trained with mean
 * squared error and Adam (beta1 0.9, beta2 0.999, eps 1e-8).  The paper
 * drives every SPH particle's micro-domain with its own history of
 * gradients (Sec. "Temporal Coupling Scheme", continuous-intermittent
 * coupling); the surrogate replaces that micro-domain where the members
 * agree, and the plain micro-DPD engine stays the fallback elsewhere.
 *
 * Arithmetic: every product is a BF16 x BF16 matrix product with FP32
 * accumulation on the matrix cores; the operands rounded to BF16 (round to
 * nearest even) are x, the weights, both hidden activations and the
 * gradients flowing into each product.  Pre-activations, biases, losses,
 * bias gradients and the Adam state are FP32.  Results are deterministic.
 *
 * Weights cross the ABI as FP32 host arrays, member after member, each
 * member packed as W1 (n_in x n_hidden, row-major), b1 (n_hidden),
 * W2 (n_hidden x n_hidden), b2, W3 (n_hidden x n_out), b3 (n_out).
 * ------------------------------------------------------------------------ */
typedef struct lhmm_sur lhmm_sur;

typedef struct {
    int32_t n_members; /* 1 .. 64                                            */
    int32_t n_in;      /* >= 1 (padded internally to a multiple of 32)       */
    int32_t n_hidden;  /* positive multiple of 32                            */
    int32_t n_out;     /* 1 .. 32                                            */
    int32_t max_batch; /* largest B of any later call                        */
} lhmm_sur_params;

/* Number of history samples of the surrogate features and the feature count
 * (4 gradient components per sample plus the polymer fraction). */
#define LHMM_SUR_HIST 32
#define LHMM_SUR_FEATURES (4 * LHMM_SUR_HIST + 1)

/* Allocate the ensemble and load weights (host, packed as above).  stream:
 * the caller's hipStream_t; all work of the engine runs on it.  Errors:
 * ARG, HIP, OOM. */
int lhmm_sur_create(const lhmm_sur_params* p, const float* weights, void* stream, lhmm_sur** out);

/* Replace the weights (host, packed) and reset the Adam state and step
 * count.  Synchronous.  Errors: ARG (non-finite weight), HIP. */
int lhmm_sur_set_weights(lhmm_sur* s, const float* weights);

/* Copy the FP32 master weights to host (packed).  Synchronous. */
int lhmm_sur_get_weights(lhmm_sur* s, float* weights);

/* Copy the gradients of the mean squared error computed by the last
 * lhmm_sur_train_step (before its update) to host, packed like the weights
 * (zeros before the first step).  A data-parallel trainer sums these across
 * replicas.  Synchronous. */
int lhmm_sur_get_grads(lhmm_sur* s, float* grads);

/* One Adam step of every member on the same minibatch.
 *   X: DEVICE B x n_in FP32 features; T: DEVICE B x n_out FP32 targets;
 *   lr: learning rate >= 0;
 *   loss: DEVICE n_members FP32, the mean squared error of each member on
 *         the minibatch before the step (NULL: not written).
 * Asynchronous.  Errors: ARG (B outside 1..max_batch), HIP. */
int lhmm_sur_train_step(lhmm_sur* s, const float* X, const float* T, int32_t B, float lr, float* loss);

/* Predictions of every member.  X: DEVICE B x n_in; Y: DEVICE
 * n_members x B x n_out.  Asynchronous.  Errors: ARG, HIP. */
int lhmm_sur_forward(lhmm_sur* s, const float* X, int32_t B, float* Y);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lhmm_sur_forward with
 * the same kernels and results, whose activations (padded BF16 inputs,
 * both hidden layers of every member, FP32 outputs) live in a 32 MiB
 * device array of the library instead of the engine's buffers.  It calls
 * no hipMalloc, hipFree or allocating routine and launches kernels only.
 * B is limited by that array, not by max_batch: Bp = B rounded up to 32
 * needs 2 Bp n_in_p + 4 n_members Bp n_hidden + 128 n_members Bp bytes
 * (n_in_p = n_in rounded up to 32, each part rounded up to 256 bytes), e.g.
 * B <= 5504 for 5 members of 129 -> 256 -> 256 -> 3; a larger B returns
 * ARG.  Call it with the device the engine was created on current (else
 * ARG).  Every call on a device shares that device's array, which keeps the
 * last call's contents: calls that overlap on one device (two streams, or
 * two threads) race and must be ordered by the caller.  X: DEVICE
 * B x n_in; Y: DEVICE n_members x B x n_out.  Asynchronous on the engine's
 * stream.  Errors: ARG, HIP. */
int lhmm_sur_forward_static(lhmm_sur* s, const float* X, int32_t B, float* Y);

/* Record sample t (t = 0, 1, ...) of the micro gradients of n particles:
 * ring is DEVICE n x LHMM_SUR_HIST x 4 FP32 (caller-owned), slot t mod
 * LHMM_SUR_HIST of particle b receives scale x (L_xx, L_xy, L_yx, L_yy) of
 * gradL (DEVICE n x 9 doubles).  stream: hipStream_t to launch on. */
int lhmm_sur_push_history(float* ring, int32_t n, const double* gradL, int64_t t, float scale, void* stream);

/* Sample t of the ring (still held: at most LHMM_SUR_HIST - 1 samples old)
 * back to traceless in-plane gradients: gradL DEVICE n x 9 doubles,
 * components / scale (inv_scale = 1 / scale).  Used to replay a particle's
 * recent history on a micro-domain. */
int lhmm_sur_history_gradient(const float* ring, int32_t n, int64_t t, float inv_scale, double* gradL, void* stream);

/* Feature rows after sample t: X (DEVICE n x LHMM_SUR_FEATURES FP32) row b
 * holds samples t-LHMM_SUR_HIST+1 .. t of particle b, oldest first, then
 * phi[b] (DEVICE n FP32, the polymer fraction of its micro-domain).  Slots
 * never written hold whatever the caller initialised the ring with. */
int lhmm_sur_features(const float* ring, int32_t n, int64_t t, const float* phi, float* X, void* stream);

/* Ensemble gate.  Y: DEVICE n_members x B x n_out (as lhmm_sur_forward
 * writes it); mean: DEVICE B x n_out, the member mean; flag: DEVICE B,
 * 1 where the spread sqrt(mean over outputs of the member variance)
 * exceeds threshold x max(|mean|_2, floor), else 0. */
int lhmm_sur_gate(const float* Y, int32_t n_members, int32_t B, int32_t n_out, float threshold, float floor,
                  float* mean, uint32_t* flag, void* stream);

/* Training targets from micro stresses: sigma DEVICE n x 6 doubles (xx, yy,
 * zz, xy, xz, yz); T DEVICE n x 3 FP32 = inv_scale x (sigma_xx - tr/3,
 * sigma_xy, sigma_yy - tr/3), the in-plane deviatoric stress the macro
 * momentum equation takes from the micro-domain (Eq. pip). */
int lhmm_sur_targets(const double* sigma, int32_t n, float inv_scale, float* T, void* stream);

/* Stress handed to the macro solver, DEVICE n x 6: row b is sigma_dpd[b]
 * where use_dpd[b] != 0 (DEVICE n uint32, NULL: none), else the traceless
 * tensor with in-plane deviatoric part scale x mean[b] (DEVICE n x 3 FP32,
 * the surrogate's (xx, xy, yy)). */
int lhmm_sur_blend(const float* mean, const uint32_t* use_dpd, const double* sigma_dpd, int32_t n, float scale,
                   double* sigma_out, void* stream);

/* Symmetry images of training samples, in place: X DEVICE n x
 * LHMM_SUR_FEATURES, T DEVICE n x 3 (xx, xy, yy).  Row b is mapped by the
 * in-plane orthogonal matrix Q = Rot(theta[b]) M, M = diag(1, -1) where
 * mirror[b] != 0 else the identity: each gradient sample L -> Q L Q^T and
 * the stress S -> Q S Q^T (the micro model is isotropic).  theta (FP32) and
 * mirror (uint32) are DEVICE n arrays of random draws supplied by the
 * caller. */
int lhmm_sur_augment(float* X, float* T, int32_t n, const float* theta, const uint32_t* mirror, void* stream);

/* Release every resource (waits for the stream).  NULL ok. */
int lhmm_sur_destroy(lhmm_sur* s);

/* ------------------------------------------------------------------------
 * The LHMM macro step with the surrogate in the loop (exchange interval of
 * the coupling protocol, one SPH step per interval, continuous-intermittent
 * micro-domains).  Per step: SPH step with the stresses of the last
 * interval; each mobile particle's micro gradient enters its history ring;
 * in LHMM_HYBRID_SURROGATE mode the ensemble predicts the deviatoric stress
 * and the gate flags particles whose members disagree or (max_grad > 0)
 * whose gradient lies outside the given input range; a flagged particle
 * runs plain micro-DPD for the next `hold` steps.  A particle entering DPD
 * without a live box gets its micro-domain back from the equilibrated
 * snapshot taken at create time and replays its last `replay` gradient
 * samples (k_micro micro steps each) before the interval, so the polymer
 * memory of its box matches its history.  Boxes on DPD advance k_micro steps
 * and their mean stress is used for their particles; the others take the
 * surrogate's mean.  With a warm band (warm_frac > 0) the boxes of unflagged
 * particles whose |L| lies in the band advance too, unused, and start from
 * the snapshot without replay when they join.  In LHMM_HYBRID_DPD mode every
 * box runs every step (the reference run).  In both modes a box whose cell
 * became thin (LHMM_FLAG_THIN) is restored and replayed the same way after
 * its stress has been used (a warming box: restored only).
 *
 * The SPH, micro and surrogate engines must share one stream; the micro
 * engine holds one box per mobile SPH particle and must already be
 * equilibrated (create takes its snapshot).  The surrogate must map
 * LHMM_SUR_FEATURES features to 3 outputs with max_batch >= the mobile
 * count.  The hybrid borrows the engines; destroy it before them.
 * ------------------------------------------------------------------------ */
typedef struct lhmm_hybrid lhmm_hybrid;

#define LHMM_HYBRID_SURROGATE 0
#define LHMM_HYBRID_DPD 1

typedef struct {
    int32_t mode;       /* LHMM_HYBRID_SURROGATE or LHMM_HYBRID_DPD          */
    int32_t k_micro;    /* micro steps per macro step (>= 1)                  */
    int32_t hold;       /* steps a flagged particle stays on DPD (>= 1)       */
    int32_t replay;     /* history samples replayed on entry or reset
                           (0 .. LHMM_SUR_HIST - 1)                           */
    float threshold;    /* gate threshold on the relative ensemble spread     */
    float floor;        /* gate floor on |mean| (surrogate output units)      */
    float grad_scale;   /* history holds L x grad_scale                      */
    float stress_scale; /* deviatoric stress = surrogate output x this       */
    float max_grad;     /* input-range gate: a particle whose micro gradient
                           L has Frobenius norm above this is flagged too
                           (the ensemble's spread does not grow where all
                           members extrapolate alike); 0 disables it        */
    float warm_frac;    /* warm band (with max_grad > 0; 0 disables it): a
                           particle whose |L| lies above warm_frac x
                           max_grad but is not flagged keeps its box live
                           on DPD without using its stress, so that a later
                           flag finds the box's memory built (no replay);
                           0 <= warm_frac <= 1                              */
} lhmm_hybrid_params;

typedef struct {
    int64_t macro_step;      /* steps done                                    */
    int64_t micro_box_steps; /* micro steps x boxes run so far, with replays  */
    int32_t n_dpd;           /* particles on DPD in the last step             */
    int32_t n_entered;       /* of which entered DPD in it                    */
    int32_t n_flagged;       /* gate flags in it                              */
    int32_t n_reset;         /* thin boxes restored after it                  */
    int32_t n_out_of_range;  /* flags of the input-range gate in it           */
    int32_t n_warm;          /* boxes advanced in the warm band in it         */
} lhmm_hybrid_stats;

/* phi: HOST n_mobile FP32, the polymer-fraction feature of each
 * particle's micro-domain.  sur may be NULL in LHMM_HYBRID_DPD mode.
 * Synchronous.  Errors: ARG, OOM, HIP, STATE (micro state not loaded). */
int lhmm_hybrid_create(const lhmm_hybrid_params* p, lhmm_sph* sph, lhmm_micro* micro, lhmm_sur* sur,
                       const float* phi, lhmm_hybrid** out);

/* One macro step; stats (HOST, may be NULL) receives its counters.  Waits
 * for the gate flags and the micro flags (two host synchronisations). */
int lhmm_hybrid_step(lhmm_hybrid* h, lhmm_hybrid_stats* stats);

/* HOST copies of the stress handed to the SPH step of the next interval
 * (n x 6; wall rows zero) and of the DPD mask of the last step (n_mobile);
 * either may be NULL.  Synchronous. */
int lhmm_hybrid_state(lhmm_hybrid* h, double* sigma, uint32_t* on_dpd);

/* HOST n x 6: the mean of the stresses handed to the SPH steps since
 * create or the last reset (may be NULL); reset != 0 restarts the mean.
 * Synchronous. */
int lhmm_hybrid_mean_stress(lhmm_hybrid* h, double* sigma_mean, int32_t reset);

int lhmm_hybrid_destroy(lhmm_hybrid* h);

/* Message of the last failing call on this thread ("" if none). */
const char* lhmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LHMM_H */
