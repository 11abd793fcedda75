/*
 * nbody.h - C interface of the MI355X library for the hot path of the hybrid symplectic
 * planetesimal integrator (Grimm & Stadel, "Terrestrial planet formation in the era of GPU
 * computing", section "The hybrid symplectic integrator").
 *
 * The method splits the Hamiltonian in democratic heliocentric coordinates (heliocentric
 * positions r_i, barycentric velocities v_i) as H = H_A + H_B + H_C (equations Ha, Hb, Hc):
 *   H_A  Kepler motion of every body about the central mass m0 (the "drift"),
 *   H_B  the all-pairs mutual gravity weighted by a smooth changeover K(r_ij) (the "kick"),
 *   H_C  the total-momentum term (the "jump"),
 * and flags pairs closer than the critical radius of equation rcrit as close encounters.
 * Beyond the plain step (nbody_step) the library integrates the close-encounter part of H_A for
 * groups of close pairs (nbody_step_hybrid: direct integration, intermediate changeover levels,
 * collisions as perfect mergers), advances ensembles of systems in one launch
 * (nbody_step_batched), picks the fastest path for small systems (nbody_step_auto), and
 * differentiates the step (nbody_*_vjp).
 *
 * Conventions shared by every entry point
 *   - Return value: NBODY_OK (0) or a negative NBODY_E_* code; the message of the last failure
 *     is available from nbody_last_error(ctx).
 *   - Every array argument is a DEVICE pointer unless stated otherwise, caller-owned, aligned to
 *     32 bytes. The library never frees caller memory; the context owns a private workspace
 *     that grows on demand (the only allocations the library makes).
 *   - Body arrays are row-major [n][4] binary64:
 *        xm  = {x, y, z, m}   heliocentric position and mass,
 *        v   = {vx, vy, vz, pad}  barycentric velocity (pad is ignored and preserved),
 *        thr = {rc, H, V, T}  per-body critical radius and encounter thresholds (see
 *                              nbody_rcrit).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and runs
 *     asynchronously. Calls on one context must not overlap: they share its workspace.
 *   - Units are the caller's; G is a parameter. Arithmetic is IEEE binary64 with
 *     round-to-nearest-even unless the split-precision kick is selected.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_OK 0
#define NBODY_E_INVAL (-1)   /* bad argument: n <= 0, NULL where required, misalignment, bad params */
#define NBODY_E_HIP (-2)     /* HIP runtime or launch failure */
#define NBODY_E_NOMEM (-3)   /* workspace allocation failed */

#define NBODY_PREC_F64 0     /* the kick entirely in binary64 */
#define NBODY_PREC_SPLIT 1   /* offsets and r^2 in binary64, r^-3 in binary32, sums in binary64 */

typedef struct nbody_params {
  double G;    /* gravitational constant */
  double m0;   /* central mass */
  double dt;   /* full step used by nbody_step and by the velocity term of rcrit */
  double n1;   /* Hill-radius factor of eq. rcrit (3) */
  double n2;   /* velocity factor of eq. rcrit (0.4) */
  double f_in; /* changeover: K = 0 below f_in * rc (0.1) */
  int32_t precision; /* NBODY_PREC_F64 or NBODY_PREC_SPLIT, used by nbody_kick / nbody_step */
  int32_t reserved;
} nbody_params;

typedef struct nbody_ctx nbody_ctx;

/* Context: parameters, workspace, autotuning table, last error. `out` is a host pointer. */
int nbody_create(nbody_ctx **out, const nbody_params *p);
int nbody_destroy(nbody_ctx *ctx);
int nbody_set_params(nbody_ctx *ctx, const nbody_params *p);
const char *nbody_last_error(const nbody_ctx *ctx);
const char *nbody_version(void);

/*
 * Workspace reservation. The context's workspace grows on demand, and growing it waits for the
 * whole device (hipDeviceSynchronize) before the old block is freed. nbody_reserve sizes it in
 * advance for systems of up to n bodies, so that later calls of that size enqueue their work
 * without allocating or synchronizing. what = a bitwise OR of
 *   NBODY_RESERVE_KICK  partial sums and momentum of nbody_kick / nbody_step / nbody_bench_pairs,
 *   NBODY_RESERVE_LIST  encounter emission (nbody_encounters, nbody_step with a list or counts),
 *   NBODY_RESERVE_CE    the close-encounter part acc_ce of nbody_kick.
 * Sizes depend on n and on the "target_waves" and "emit_slots" tuning values at the time of the
 * call. Synchronizes `stream` before returning. Returns NBODY_E_INVAL for unknown flags,
 * NBODY_E_NOMEM if the device memory is not available.
 */
#define NBODY_RESERVE_KICK 1u
#define NBODY_RESERVE_LIST 2u
#define NBODY_RESERVE_CE 4u
int nbody_reserve(nbody_ctx *ctx, int64_t n, uint32_t what, void *stream);

/*
 * Critical radius and encounter thresholds (eq. rcrit), one row per body:
 *   rc_i = max(n1 R_Hill,i, n2 dt |v_i|),  R_Hill,i = |x_i| (m_i / (3 m0))^(1/3),
 *   H_i  = cH * ((r2_i*r2_i)*r2_i) * (mu_i*mu_i),  cH = ((n1*n1*n1)*(n1*n1*n1))/9, mu_i = m_i/m0,
 *          r2_i = fma(z,z,fma(y,y,x*x))            [ = (n1 R_Hill,i)^6 ],
 *   V_i  = cV * fma(vz,vz,fma(vy,vy,vx*vx)),  cV = (n2*dt)*(n2*dt)   [ = (n2 dt |v_i|)^2 ],
 *   T_i  = an upper bound of every r^2 that the thresholds of body i can flag (internal).
 * thr [n][4] is written. The step functions hold thr fixed for a whole call.
 */
int nbody_rcrit(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, double *thr,
                void *stream);

/*
 * H_B kick (eq. Hb): the gradient of -sum_{i<j} G m_i m_j K(r_ij)/r_ij with rc held fixed,
 *   a_i = G sum_{j != i} m_j w_ij (x_j - x_i),
 *   w = 1/r^3 for pairs that are not close, w = K/r^3 - K'(r)/r^2 for close pairs, with
 *   K(y) = y^2/(2y^2-2y+1), y = clamp((r - f_in rc_ij)/((1-f_in) rc_ij), 0, 1),
 *   rc_ij = max(rc_i, rc_j), and "close" the exact predicate of nbody_encounters.
 * v (in/out, may be NULL): v_i += h a_i.  acc [n][4] (may be NULL): a_i.  acc_ce [n][4] (may be
 * NULL): the complementary close-encounter part G sum_close m_j (1/r^3 - w) (x_j - x_i), so that
 * acc + acc_ce is the plain Newtonian pull. Precision follows params.precision.
 */
int nbody_kick(nbody_ctx *ctx, int64_t n, const double *xm, const double *thr, double *v, double h,
               double *acc, double *acc_ce, void *stream);

/*
 * nbody_kick without allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kick and outputs
 * as nbody_kick, with its workspace (partial sums, equal-mass flag) in a 32 MiB device array
 * the library holds per device until the process ends, instead of the context's workspace. It
 * calls no allocating routine. Sizes whose workspace exceeds the array (n above about 1e6, or
 * about 5e5 with acc_ce) are rejected with NBODY_E_INVAL. The j-chunk count may be lower than
 * nbody_kick's, so sums may differ from it in the last bits. Calls that overlap on one device
 * (other streams or threads) share the array and race.
 */
int nbody_kick_noalloc(nbody_ctx *ctx, int64_t n, const double *xm, const double *thr, double *v,
                       double h, double *acc, double *acc_ce, void *stream);

/*
 * Close-encounter pairs (the pairs inside the critical radius, eq. rcrit): i < j with
 *   (r2*r2)*r2 < max(H_i, H_j)  or  r2 < max(V_i, V_j),
 *   r2 = fma(dz,dz,fma(dy,dy,dx*dx)), d = x_j - x_i,
 * evaluated exactly in binary64 (in real arithmetic: r_ij < max(rc_i, rc_j)).
 * pairs [cap][2] int32 receives the first min(count, cap) pairs in ascending (i, j) order;
 * *count (device int64) receives the true number of pairs, so count > cap signals truncation.
 */
int nbody_encounters(nbody_ctx *ctx, int64_t n, const double *xm, const double *thr,
                     int32_t *pairs, int64_t cap, int64_t *count, void *stream);

/* H_C jump (eq. Hc): x_i += h * (P / m0) with P = sum_j m_j v_j. xm in/out, v read. */
int nbody_jump(nbody_ctx *ctx, int64_t n, double *xm, const double *v, double h, void *stream);

/*
 * H_A drift (eq. Ha, first line): every body moves for time h along its Kepler orbit about
 * mu = G m0 (universal-variable formulation, binary64). xm (positions) and v in/out.
 * status [n] uint32 (may be NULL): 0, or 1 if the anomaly iteration did not converge.
 */
int nbody_drift(nbody_ctx *ctx, int64_t n, double *xm, double *v, double h, uint32_t *status,
                void *stream);

/*
 * nsteps steps B(dt/2) C(dt/2) A(dt) C(dt/2) B(dt/2). thr: NULL = computed from the state at
 * call start into the context; otherwise used as given. thr is held fixed for the call, so a
 * call is exactly the composition of its steps and consecutive kicks at the same positions are
 * evaluated once (v += h a applied twice). If count is not NULL the encounter list at the final
 * positions is written to pairs/cap/count as in nbody_encounters. step_counts (device int64
 * [nsteps + 1], may be NULL) receives the number of close pairs (same predicate) at each of the
 * nsteps + 1 force evaluations: the initial positions, then the positions of each step's second
 * kick; the counts come from the kick's own pair loop.
 */
int nbody_step(nbody_ctx *ctx, int64_t n, double *xm, double *v, const double *thr, int32_t nsteps,
               int32_t *pairs, int64_t cap, int64_t *count, int64_t *step_counts, void *stream);

/*
 * Close-encounter groups: the connected components of the graph whose edges are the close pairs,
 * i.e. the sets of bodies that the hybrid method's close-encounter integration has to treat
 * together (section "The hybrid symplectic integrator"). The edges are the first min(*count, cap)
 * entries of pairs [cap][2] (device int32; count device int64), as written by nbody_encounters
 * or nbody_step. labels [n] (device int32) receives for every body the smallest body index of its
 * group (a body without close partners is its own group). out (device int64 [2]) receives
 * {number of groups with at least two bodies, number of pairs ignored because an index lies
 * outside 0..n-1 or i == j}. Lock-free union-find; the labels are unique, so the result does not
 * depend on thread timing.
 */
int nbody_encounter_groups(nbody_ctx *ctx, int64_t n, const int32_t *pairs, int64_t cap,
                           const int64_t *count, int32_t *labels, int64_t *out, void *stream);

/*
 * Collisions as perfect mergers (the outcomes of collisions, in the paper's section on further
 * physics, with the radius factor f of its section on the acceleration factor), applied inside the
 * close-encounter drift. Two bodies of a group are in contact when their distance falls below
 * f (R_i + R_j). The drift finds the first contact time (the first integrator step that ends in
 * contact, then bisection on that step's length) and merges the pair there: the lower body index
 * keeps the summed mass, the summed volume (R^3 = R_i^3 + R_j^3) and the centre-of-mass position
 * and velocity; the other body becomes massless with zero radius and is parked on a circular
 * orbit of radius 1e6 about the central mass at the angle 2 pi j/n, where it meets nothing (callers
 * may drop such bodies between calls). Contacts are looked for only within groups: with rc far above
 * f R a colliding pair is a close pair at the start of the step.
 *   radius  device double [n]: physical radii, in/out (merged bodies updated, removed ones 0).
 *   f       radius factor, finite and >= 0 (0: no contact is possible).
 *   merges  device int32 [cap][3]: {step within the call, survivor, removed} per merger, in no
 *           particular order; time: device double [cap], the time of each merger within its step's
 *           drift. Both may be NULL when cap is 0.
 *   count   device int64: number of mergers in the call (set to 0 first; may exceed cap, in which
 *           case only cap are logged).
 * Ownership stays with the caller; all pointers are device pointers.
 */
typedef struct nbody_collisions {
  double *radius;
  double f;
  int32_t *merges;
  double *time;
  int64_t cap;
  int64_t *count;
} nbody_collisions;

/*
 * Close-encounter drift: H_A in full (eq. Ha, both lines) over time h. The bodies of every
 * close-encounter group (labels as written by nbody_encounter_groups: the smallest index of each
 * body's group) move under the equations of motion of H_A restricted to their group,
 *   dx_i/dt = v_i,
 *   dv_i/dt = -G m0 x_i/|x_i|^3 + G sum_{j in group, j != i} m_j ((1 - K)/r^3 + K'(r)/r^2) d_ij,
 * integrated with the Gragg-Bulirsch-Stoer method (binary64, tolerance 1e-14 relative to the
 * group's largest position and velocity), one workgroup of four waves per group (the waves run
 * the extrapolation's midpoint sweeps side by side); a body alone in its group follows its Kepler
 * orbit (as nbody_drift). thr as from nbody_rcrit (rc_i sets the changeover).
 * col (may be NULL): collisions as perfect mergers within the groups (see nbody_collisions).
 * stats (device int64 [6]) receives: [0] groups integrated, [1] largest group, [2] bodies in
 * groups, [3] groups of more than 64 bodies (moved on Kepler orbits only: the result is then not
 * the H_A flow, and no contacts are found in them), [4] groups whose integration did not finish,
 * [5] (nbody_step_hybrid only) encounter lists that exceeded the internal capacity of
 * max(16 n, 65536) pairs (the groups of that evaluation were built from the first pairs only).
 * Non-zero [3], [4] or [5] mean that part of the result is not the method's; the call still
 * returns NBODY_OK (the state is valid), and the Python binding raises a warning for each.
 */
int nbody_drift_groups(nbody_ctx *ctx, int64_t n, double *xm, double *v, const double *thr,
                       const int32_t *labels, double h, const nbody_collisions *col, int64_t *stats,
                       void *stream);

/*
 * Multi-level changeover (the paper's intermediate levels between the symplectic step and the
 * direct close-encounter integrator, section "The hybrid symplectic integrator"). Level l has the
 * time step dt / substeps^l and critical radii from eq. rcrit at that step (thresholds taken at
 * the call's start). The drift of the bodies with close partners integrates
 * H_A = Kepler + W_0 U over the step's close pairs (U = -G m_i m_j / r, W_l = prod_{i<=l} [1 - K_i]);
 * above the deepest level L a level-l drift over tau is substeps substeps of
 * kick(tau/2s) drift_{l+1}(tau/s) kick(tau/2s), the kick acting on the close pairs with the
 * potential W_l K_{l+1} U; at level L the close pairs still within rc_L form the groups that the
 * direct integrator takes (pair term weighted by W_L), and the other bodies follow Kepler orbits.
 * levels = 0 is the plain hybrid step; at most 4 levels. margin (finite, >= 0): with levels, the
 * step's close-pair list is taken at (1 + margin) rc (exact-predicate thresholds H (1+margin)^6,
 * V (1+margin)^2; the kick is unchanged, as K = 1 beyond rc), so that pairs which cross rc during the
 * step are integrated by the drift; 0.5 keeps the full energy of the 32768-body disk to 1e-11 over
 * 10 steps where 0 drifts by 2e-9.
 */
typedef struct nbody_levels {
  int32_t levels;
  int32_t substeps;
  double margin;
} nbody_levels;

/*
 * Hybrid step: as nbody_step (B(dt/2) C(dt/2) A(dt) C(dt/2) B(dt/2), thresholds fixed for the
 * call, merged half kicks), but the drift A integrates H_A in full: the close pairs found by each
 * kick's pair loop form the close-encounter groups of the drift that follows, integrated as in
 * nbody_drift_groups. The step then conserves the full energy E instead of the K-weighted E'.
 * n bodies; xm, v as for nbody_step; thr as from nbody_rcrit, or NULL (computed at the call's
 * start); nsteps >= 0. lv (may be NULL: no intermediate levels): multi-level changeover (see
 * nbody_levels; levels outside 0..4 or substeps < 1 are rejected); contacts are then looked for by
 * the direct integrator at the deepest level and merger times are within that level's substep.
 * col (may be NULL): collisions as perfect mergers in every step's drift (merged masses take part
 * in the kicks that follow; rc stays fixed for the call). stats (device int64 [6]) as for
 * nbody_drift_groups, summed over the steps (stats[1] the maximum). Binary64 only: a context in
 * split precision is rejected. Returns NBODY_OK, NBODY_E_INVAL, NBODY_E_NOMEM or NBODY_E_HIP.
 */
int nbody_step_hybrid(nbody_ctx *ctx, int64_t n, double *xm, double *v, const double *thr,
                      int32_t nsteps, const nbody_levels *lv, const nbody_collisions *col,
                      int64_t *stats, void *stream);

/*
 * Small-N switch. The paper notes that small systems leave a GPU idle, dominated by per-kernel
 * overhead, and that self-tuning routines pick the fastest integration setup for a problem size
 * (section "The GENGA code"). Here a single system advances either with nbody_step's per-step
 * launches (path 0) or in one persistent launch of the ensemble kernel of nbody_step_batched
 * (paths 1 and 2: its group and wave tiles; binary64, n <= 2048, resp. n <= 256), which removes the
 * launch latency per step; the two agree to about 1e-12 relative, not bit for bit.
 * nbody_autotune_step times every admissible path for ntrial steps on scratch copies of (xm, v)
 * (inputs unchanged), records the fastest for this n in the context, and writes it to *choice
 * (host int32, may be NULL). It synchronizes the stream.
 */
int nbody_autotune_step(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, int32_t ntrial,
                        int32_t *choice, void *stream);

/*
 * nsteps steps of one system of n bodies in place with the path recorded for n by
 * nbody_autotune_step (path 0, identical to nbody_step with thr = NULL, if n was never tuned, or
 * when the context's precision is not binary64). Thresholds are taken at the call's start.
 * nbody_set_params forgets the recorded paths.
 */
int nbody_step_auto(nbody_ctx *ctx, int64_t n, double *xm, double *v, int32_t nsteps, void *stream);

/*
 * Input check before integrating a state. The method has no softening, so a body at the central
 * mass (r_i = 0 in eq. Ha) or two bodies at one position (r_ij = 0 in eq. Hb) are invalid input.
 * result (device int64 [2]) receives {i, reason} for the smallest body index i with a problem
 * (and the smallest reason code for that index), or {-1, 0}:
 *   1 = a non-finite position, mass or velocity component;   2 = negative mass;
 *   3 = position exactly at the central mass;                4 = same position as a body j > i.
 * The coincidence test is an all-pairs scan (about the cost of one kick). Deterministic.
 */
int nbody_validate(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, int64_t *result,
                   void *stream);

/*
 * Diagnostics (device out[8]): E (full Newtonian energy in democratic heliocentric form),
 * E' (the pair term weighted by K: the quantity the hot-path step conserves), L[3], P[3].
 */
int nbody_energy(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, const double *thr,
                 double *out, void *stream);

/*
 * Launch-shape tuning of a context (host values; results never depend on them except where
 * stated): "locality_min_n" (bodies from which the pair kernels group spatially close bodies
 * into waves, default 4096; this changes no result bit), "locality_every" (steps between
 * regroupings inside nbody_step, default 10), "emit_slots" (upper bound of the partner slots per
 * row and j-chunk before a row is rescanned, default 64), "target_waves" (waves per pair-kernel
 * launch, default 32768; changes the summation order of the j-chunks). Returns NBODY_E_INVAL for an unknown key
 * or a value out of range.
 */
int nbody_tune(nbody_ctx *ctx, const char *name, int64_t value);

/*
 * Batched ensembles: nsys independent systems, each a central mass m0 with its own bodies, all
 * advanced by nsteps steps of nbody_step (thresholds from each system's initial state, binary64)
 * in ONE persistent launch. System s occupies rows offs[s] .. offs[s+1]-1 of xm and v; offs is a
 * HOST array of nsys+1 int64 with offs[0] = 0 and 1 <= offs[s+1]-offs[s] <= 2048. npairs
 * (device uint64 [nsys], may be NULL) receives each system's number of close pairs at its final
 * positions. Workgroups take systems largest first; the tile used for a system (one workgroup
 * or one wave per system, one or two bodies per lane) comes from the context's table of size
 * classes (N <= 64, 128, 256, 512, 1024, 2048). The result of a system depends only on its own bodies and its tile, not on
 * the rest of the ensemble. The call returns when the work is complete.
 */
int nbody_step_batched(nbody_ctx *ctx, int32_t nsys, const int64_t *offs, double *xm, double *v,
                       int32_t nsteps, uint64_t *npairs, void *stream);

/*
 * Autotuner of the batched tiles ("self-tuning routines", section "The GENGA code"). A tile code
 * is a bit set: bit 0 set = one wave per system (applies to systems of at most 256 bodies; larger
 * ones run as if it were clear), clear = one workgroup (eight waves) per system; bit 1 set = each
 * lane of the kick owns two bodies (one j-body read serves two pairs), clear = one. Codes 0 .. 3.
 * Every class present is timed on its own systems (the others skipped) for nsteps steps (on
 * scratch copies; xm and v are not modified) with each admissible code, in order and then in
 * reverse order; another code replaces the current one only if it is more than 2 % faster. The
 * resulting table is then timed on the whole ensemble against each code applied to every class
 * (without the wave bit where a class cannot take it), again in symmetric order and with the
 * same 2 % margin, because the classes share the launch's queue. Use nsteps of 10 or more: very
 * short runs favour the wave tile. get/set read or replace the table (host array of 6 codes); get
 * returns the number of classes.
 */
int nbody_autotune_batched(nbody_ctx *ctx, int32_t nsys, const int64_t *offs, const double *xm,
                           const double *v, int32_t nsteps, void *stream);
int nbody_get_batched_tiles(const nbody_ctx *ctx, int32_t *tiles, int32_t n);
int nbody_set_batched_tiles(nbody_ctx *ctx, const int32_t *tiles, int32_t n);

/*
 * Reverse-mode derivatives (vector-Jacobian products) with the thresholds thr held fixed, for
 * sensitivity analysis and orbit fitting. Adjoint arrays mirror the state layout:
 * lam_x [n][4] = dL/d{x, y, z, m} and lam_v [n][4] = dL/d{vx, vy, vz, pad}; the mass adjoint
 * accumulates in lam_x[:, 3]. All adjoint arrays are device, in/out.
 *
 * nbody_kick_vjp:  for v' = v + h a(x, m) at positions xm: lam_x += (d(h a)/d(x, m))^T lam_v
 *                  (lam_v itself passes through unchanged).
 * nbody_jump_vjp:  for x' = x + h P/m0, P = sum m_j v_j, at state (xm, v):
 *                  lam_v_j += (h/m0) m_j sum_i lam_x_i,  lam_x_j[3] += (h/m0) v_j . sum_i lam_x_i.
 * nbody_drift_vjp: for the drift by h from the state (xm, v) BEFORE the drift: replaces
 *                  (lam_x[:, 0:3], lam_v[:, 0:3]) by their pull-back through the Kepler flow.
 * nbody_step_vjp:  for nsteps steps of nbody_step starting at (xm0, v0) with thresholds thr:
 *                  on entry (lam_x, lam_v) hold dL/d(final state) (lam_x[:, 3] any accumulated
 *                  dL/dm); on return they hold dL/d(xm0, v0), lam_x[:, 3] having gained the mass
 *                  derivatives of these steps. States inside the segment are recomputed from
 *                  (xm0, v0) bit for bit; workspace grows by 2 n nsteps x 32 bytes.
 */
int nbody_kick_vjp(nbody_ctx *ctx, int64_t n, const double *xm, const double *thr, double h,
                   const double *lam_v, double *lam_x, void *stream);
int nbody_jump_vjp(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, double h,
                   double *lam_x, double *lam_v, void *stream);
int nbody_drift_vjp(nbody_ctx *ctx, int64_t n, const double *xm, const double *v, double h,
                    double *lam_x, double *lam_v, void *stream);
int nbody_step_vjp(nbody_ctx *ctx, int64_t n, const double *xm0, const double *v0, const double *thr,
                   int32_t nsteps, double *lam_x, double *lam_v, void *stream);

/*
 * Measurement helper: launches the pair kernel of nbody_kick (no velocity update, no outputs
 * beyond the context's partial sums) `reps` times between two HIP events recorded on `stream`,
 * waits for the second event and stores the mean duration of one launch in milliseconds in
 * *avg_ms (a HOST pointer). Used to state the kernel's achieved fraction of peak.
 */
int nbody_bench_pairs(nbody_ctx *ctx, int64_t n, const double *xm, const double *thr, int32_t reps,
                      double *avg_ms, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
