/*
 * genga.h - C ABI of libgenga.so, the MI355X (gfx950) hot path of the hybrid
 * symplectic N-body method of GENGA II (Grimm et al. 2022, arXiv 2201.10058).
 *
 * Method (paper Sect. 2, eqs. H, Ha, Hb, Hc and rcrit; Appendix A): bodies
 * are held in democratic coordinates (heliocentric positions, barycentric
 * velocities).  One base step is
 *     Rcrit(dt); Kick(dt/2) + encounter pre-check; HC(dt/2); FG(dt);
 *     HC(dt/2); Kick(dt/2).
 * The kick is the interaction part H_B: every pair of bodies (not the star)
 * exchanges Newtonian gravity weighted by the changeover function
 * K(r_ij; rho_ij) of Sect. 6.2 (zero below 0.1 rho, one above rho, the
 * smooth form of Chambers 1999 eq. 10 between), with rho_ij = max(rc_i, rc_j).
 * Pairs closer than rho_ij form the close-encounter list that the direct
 * solver takes (Sect. 2; list order fixed as in Appendix B, "exact
 * reproducible results").  genga_step runs the direct solver (close-encounter
 * groups integrated by Bulirsch-Stoer extrapolation) when p->direct is set.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array pointer is a DEVICE pointer owned by the caller
 *   (contiguous, float64 structure-of-arrays of length n unless stated).  The
 *   library never allocates device memory in a call: scratch space is the
 *   caller's workspace `ws` of genga_workspace_bytes() bytes, 256-byte
 *   aligned; a new workspace is zero-filled by the caller (or passed to
 *   genga_clear_status) before its first use, so that its status word starts
 *   clear.  Host-side structs (genga_bodies, genga_params, genga_pairs) are
 *   read during the call only and may be freed on return.
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *   enqueued asynchronously in order on that stream; results are valid after
 *   the stream is synchronised.  Calls that share a workspace must be ordered
 *   on one stream.
 * Errors.  Argument errors are detected on the host and returned at once
 *   (GENGA_E_INVAL), with nothing enqueued.  Errors found by kernels (encounter
 *   list overflow, coincident bodies, non-finite results, invalid critical
 *   radii, Kepler solver failure) set bits in a status word inside the
 *   workspace; genga_read_status() synchronises the stream, returns the most
 *   severe code and clears the word.  genga_step() reads it itself unless
 *   GENGA_FLAG_NOSYNC is set.
 * Determinism.  Every kernel is free of floating-point atomics; sums run in a
 *   fixed order for a fixed launch configuration, so repeated calls with the
 *   same inputs give bitwise identical results.  The encounter list is always
 *   produced in canonical order (i ascending, then j ascending, i < j).
 */
#ifndef GENGA_H
#define GENGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define GENGA_OK             0
#define GENGA_E_INVAL       (-1) /* null pointer, n < 1, non-finite scalar, bad size  */
#define GENGA_E_OVERFLOW    (-2) /* more encounter pairs than capacity (count is true) */
#define GENGA_E_NONFINITE   (-3) /* two distinct bodies coincide, or a NaN/inf result  */
#define GENGA_E_HIP         (-4) /* a HIP runtime call failed (genga_last_hip_error)   */
#define GENGA_E_UNSUPPORTED (-5) /* option not available on this device               */
#define GENGA_E_NOCONV      (-6) /* Kepler solver or Bulirsch-Stoer did not converge    */
#define GENGA_E_RCRIT       (-7) /* a critical radius is negative or NaN               */
#define GENGA_E_GROUP       (-8) /* a close-encounter group exceeds the direct solver's
                                    GENGA_GROUP_MAX bodies (its bodies kept their drift) */
#define GENGA_E_SCRATCH     (-9) /* genga_kick_static: the problem needs more scratch
                                    than GENGA_STATIC_SCRATCH_BYTES                 */

/* genga_params.precision */
#define GENGA_FP64  0 /* all pair arithmetic in binary64                              */
#define GENGA_MIXED 1 /* binary32 pair arithmetic on binary64 differences, binary64
                         accumulation, binary64 encounter test (see genga_kick)       */

/* genga_params.flags */
#define GENGA_FLAG_NOSYNC 1 /* genga_step: do not synchronise nor read the status     */
/* Form of the kick (Newton's third law, Sect. 2: the pair
 * force and its changeover weight K(r_ij; max(rc_i, rc_j)) are symmetric in i
 * and j).  The symmetric form evaluates each unordered pair once and applies
 * it to both bodies; the one-sided form evaluates every ordered pair for its
 * first body.  Both give the same encounter list (bit for bit) and
 * accelerations that differ by summation order only.  By default the
 * symmetric form runs from n >= 8192 bodies (up to about 370,000: its
 * workspace holds row and column sums that grow as n^2 / 512, 8 GiB there,
 * 0.34 GiB at 65,536 bodies) in the all-massive kick, binary64
 * and mixed (genga_kick, genga_step and the levels' base kick), and in the
 * binary64 batch (genga_kick_batched, genga_step_batched; every system, in
 * 512-row groups and 512-column slices); the flags force one form at any n
 * (both set: GENGA_E_INVAL).  Test-particle modes, the mixed batch and
 * genga_encounter_pairs are one-sided whatever the flags. */
#define GENGA_FLAG_DIRECTED  2
#define GENGA_FLAG_SYMMETRIC 4

/* Bodies of one system, democratic coordinates, device SoA of length n.
 * rc holds the critical radii r_crit,i (eq. rcrit); genga_rcrit writes it.    */
typedef struct {
    int64_t n;
    double *x, *y, *z;    /* heliocentric positions [AU]                        */
    double *vx, *vy, *vz; /* barycentric velocities [AU/day]                    */
    double *m;            /* masses [solar masses]; the star is not an element  */
    double *rc;           /* critical radii [AU], >= 0                          */
    double *R;            /* physical radii [AU] (nullable): with the direct
                             solver, members closer than R_i + R_j merge (see
                             genga_step); mergers update m and R            */
} genga_bodies;

/* Scalars of the method.  Units are the caller's; G must match them. */
typedef struct {
    double G;      /* gravitational constant                                    */
    double m_star; /* central mass (H_A Kepler term and H_C)                    */
    double dt;     /* base time step (eq. rcrit and genga_step)                 */
    double n1;     /* Hill-radius factor of eq. rcrit (paper: 3)                */
    double n2;     /* velocity factor of eq. rcrit (paper: 0.4)                 */
    int precision; /* GENGA_FP64 or GENGA_MIXED                                 */
    int flags;     /* GENGA_FLAG_*                                              */
    int ipt;       /* kick rows per thread (1 or 2); 0 = library choice         */
    int slices;    /* single system: kick column slices; 0 = library choice.
                      Symmetric kick: slices of 512 / d columns with d the
                      largest power of two <= min(slices, 8) (a binary64
                      batch: <= min(slices, 4); 0 = the width whose tiles
                      finish first by the batch plan's schedule model)     */
    int block;     /* batch: kick threads per block (64 or 256); 0 = 256         */
    int tile_cols; /* batch: columns per kick tile (rounded up to 64); 0 = 1024  */
    int grid;      /* batch: persistent kick blocks; 0 = library choice         */
    void *prof_events[4]; /* optional hipEvent_t handles (timing): [0], [1] are
                             recorded immediately before and after the main
                             kernel of genga_kick and of the first half kick of
                             genga_step; [2], [3] around the second half kick
                             of genga_step.  NULL entries are skipped.        */
    int tp_mode;   /* test-particle mode (Sect. 8): bodies [0, n_massive) are
                      massive, [n_massive, n) test particles, which never act
                      on each other.  0: every body acts on every other (the
                      default; n_massive ignored).  1: test particles feel the
                      massive bodies but act on nothing (they are left out of
                      the HC momentum too).  2 (semi-active): as 1, but test
                      particles act on the massive bodies as in mode 0.  The
                      encounter list then holds the pairs whose first body is
                      massive.  Modes 1 and 2 run in the binary64 single-system
                      genga_kick, genga_encounter_pairs, genga_hc and genga_step;
                      elsewhere they return GENGA_E_UNSUPPORTED.              */
    int slevels;   /* symplectic levels of genga_step (Sect. 6.2, higher-level
                      changeover functions; Appendix A, recursive encounter
                      routine).  0 or 1: the base step.  L in [2, GENGA_MAX_LEVELS]:
                      the bodies of the level-0 encounter list are advanced,
                      instead of their drift, by `substeps` sub-steps of dt /
                      substeps at level 1, whose own encounters go one level
                      deeper, down to level L - 1 (see genga_step).         */
    int64_t n_massive; /* number of massive bodies (0 <= n_massive <= n)        */
    int substeps;  /* sub-steps per level (>= 1 when slevels > 1)               */
    int direct;    /* 1: genga_step also integrates the deepest level's
                      remainder with the direct solver (close-encounter
                      groups + Bulirsch-Stoer, Sect. 2 and Sect. 6.1; see
                      genga_step).  0: that remainder is left out.          */
    int64_t level_capacity; /* slevels > 1 or direct: pairs each level's list
                               can hold; genga_workspace_bytes sizes the
                               workspace for it.  A level-0 list longer than
                               this sets GENGA_E_OVERFLOW: the levels then used
                               only its first level_capacity pairs, and
                               genga_step's `pairs` receives those and the true
                               count.                                        */
    double bs_eps; /* direct solver: relative tolerance of the Bulirsch-Stoer
                      extrapolation; 0 = 1e-12                               */
    double c_light; /* speed of light in the caller's units: > 0 adds the
                       post-Newtonian term to genga_step (genga_gr_kick);
                       0 = off                                               */
    double coll_tol; /* collisions: contact located to an overlap below this
                        fraction of R_i + R_j (the paper's collision
                        precision); 0 = 1e-6                                 */
} genga_params;

#define GENGA_MAX_LEVELS 8
#define GENGA_GROUP_MAX 65536 /* bodies of the largest group the direct solver takes
                                 (groups above 512 bodies spread over all compute units;
                                 a device that cannot hold 256 workgroups of 256 threads
                                 at once takes correspondingly fewer)                   */

/* Close-encounter list (device memory). */
typedef struct {
    int32_t *i, *j;   /* capacity entries each; pair k is (i[k], j[k]), i < j    */
    int64_t capacity; /* entries available in i and j (may be 0)                 */
    int64_t *count;   /* one device int64: receives the TRUE number of pairs     */
} genga_pairs;

/* Library version (major * 10000 + minor * 100 + patch). */
int genga_version(void);

/* Text for a return code. */
const char *genga_strerror(int code);

/* The last hipError_t seen by the library on this thread (0 if none). */
int genga_last_hip_error(void);

/* Workspace size in bytes for systems of up to n bodies with these params.
 * Returns 0 for n < 1. */
size_t genga_workspace_bytes(int64_t n, const genga_params *p);

/* Synchronise `stream`, return the most severe status recorded in the
 * workspace since the last read (GENGA_OK if none) and clear it. */
int genga_read_status(void *ws, void *stream);

/* Clear the workspace status word (asynchronously, on `stream`). */
int genga_clear_status(void *ws, void *stream);

/* Critical radii, eq. (rcrit), paper Sect. 2:
 *   rc_i = max(n1 * R_H,i, n2 * |dt| * |v_i|),
 *   R_H,i = |x_i| * (m_i / (3 m_star))^(1/3).
 * Reads x..vz, m; writes b->rc. */
int genga_rcrit(const genga_bodies *b, const genga_params *p, void *ws, void *stream);

/* Kick: the interaction part H_B (paper Sect. 2, eq. Hb; Appendix A).
 *   a_i = G sum_{j != i} m_j K(r_ij; rho_ij) (x_j - x_i) / r_ij^3,
 *   rho_ij = max(rc_i, rc_j),  v_i += h * a_i.
 * h = 0 leaves the velocities untouched.  ax/ay/az (nullable, device, n)
 * receive a.  pairs (nullable) receives the close-encounter list of the same
 * positions: pairs with i < j and r_ij^2 < rho_ij^2, where
 * r_ij^2 = fma(dz, dz, fma(dy, dy, dx * dx)) and d = x_j - x_i in binary64
 * (the "close-encounter pre-check" of Appendix A), in canonical order.
 * If the count exceeds capacity, the first `capacity` pairs are written, the
 * true count is stored and the status records GENGA_E_OVERFLOW.
 * precision GENGA_MIXED: differences d in binary64 rounded to binary32,
 * binary32 distance, weight and partial sums over 64 columns (the symmetric
 * form's column side: over the 128 rows of a wave), folded into binary64
 * accumulators; every pair closer than 3 rho_ij (selected by a
 * conservative binary32 test) is evaluated entirely in binary64, and the
 * encounter test stays in binary64, so the list is identical to GENGA_FP64.
 * A row whose binary32 terms add up in magnitude (sum m_j / r_ij^2) to more
 * than 10 times the magnitude of their sum is evaluated again entirely in
 * binary64 (strong cancellation would otherwise magnify the binary32 term
 * errors); after the call the third int32 of the workspace holds the number
 * of such rows.
 * Positions of two distinct bodies that coincide set GENGA_E_NONFINITE. */
int genga_kick(const genga_bodies *b, const genga_params *p, double h,
               double *ax, double *ay, double *az, genga_pairs *pairs, void *ws, void *stream);

/* genga_kick without a workspace, for callers that cannot allocate device
 * memory: code under HIP graph capture that may not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, kernels
 * and results as genga_kick (bit for bit, for the same params), except:
 *  - scratch is a static device array of GENGA_STATIC_SCRATCH_BYTES bytes
 *    that the library holds on every GPU it runs on until the process ends;
 *    the call allocates nothing.  A kick that needs more (for the default
 *    shapes: more than about 9,600 bodies) returns GENGA_E_SCRATCH at once,
 *    with nothing enqueued;
 *  - status (device int32, required) receives, when the stream reaches the
 *    end of the call, GENGA_OK or the most severe code the kernels found
 *    (GENGA_E_OVERFLOW, GENGA_E_NONFINITE, GENGA_E_RCRIT).
 * Every call on one GPU shares that GPU's array and clears its status words
 * first: calls that overlap on one GPU (different streams, or host threads
 * without ordering) race and give undefined results.  The first call on a
 * device looks up the array's device address (hipGetSymbolAddress). */
#define GENGA_STATIC_SCRATCH_BYTES ((size_t)96 << 20)
int genga_kick_static(const genga_bodies *b, const genga_params *p, double h, double *ax,
                      double *ay, double *az, genga_pairs *pairs, int32_t *status, void *stream);

/* Close-encounter list alone (same predicate and order as genga_kick); used
 * for the detection after the drift (Appendix A). */
int genga_encounter_pairs(const genga_bodies *b, const genga_params *p, genga_pairs *pairs,
                          void *ws, void *stream);

/* HC, the Sun part H_C (eq. Hc):  x_i += h * P / m_star,  P = sum_j m_j v_j.
 * P is summed in a fixed order. */
int genga_hc(genga_bodies *b, const genga_params *p, double h, void *ws, void *stream);

/* FG, the Keplerian part of H_A (Sect. 2): every body follows its two-body
 * orbit about the star (mu = G m_star) for a time dt, by Gauss f and g
 * functions in the universal anomaly (elliptic and hyperbolic orbits). */
int genga_drift(genga_bodies *b, const genga_params *p, double dt, void *ws, void *stream);

/* One base step of Appendix A without the direct solver:
 *   rc <- Rcrit(x, v); Kick(dt/2) [+ pairs]; HC(dt/2); FG(dt); HC(dt/2);
 *   Kick(dt/2) with the same rc.
 * pairs (nullable) receives the list of the first half kick.  Unless
 * GENGA_FLAG_NOSYNC, synchronises the stream and returns the status.
 *
 * Symplectic levels (p->slevels = L > 1; Sect. 6.2 and Appendix A): the
 * bodies of the level-0 list E_0 are not drifted for dt; from their state
 * before the drift, level l = 1 advances them by `substeps` sub-steps of
 * dt_l = dt_{l-1} / substeps (dt_0 = dt).  Each sub-step: critical radii
 * rc_l of eq. (rcrit) with dt_l for the bodies of E_{l-1}; E_l = the pairs
 * of E_{l-1} with r^2 < max(rc_l,i, rc_l,j)^2 (canonical order); a kick of
 * dt_l / 2 over the pairs of E_{l-1} with the weight
 *   W_l(r) = prod_{k<l} (1 - K(r; rho_k)) * K(r; rho_l),
 * each pair acting on both bodies; the drift of E_{l-1}'s bodies for dt_l,
 * except that, for l < L - 1, E_l's bodies are instead advanced by level
 * l + 1 from their state before that drift; and the same kick again.  The
 * remainder prod_{k<L} (1 - K(r; rho_k)), the direct solver's part, is not
 * integrated (as for L = 1) unless p->direct.  There is no H_C term inside
 * the levels.
 *
 * Direct solver (p->direct = 1; Sect. 2 and Sect. 6.1; Appendix A "grouping"
 * and "Bulirsch-Stoer"): the deepest list D (E_0 for L = 1, else the list
 * E_{L-1} of each sub-step of level L - 1) is split into close-encounter
 * groups, the connected components of its pair graph; the bodies of each
 * group move, instead of their drift over that level's interval, under
 *   dx_i/dt = v_i,
 *   dv_i/dt = -G m_star x_i/|x_i|^3 + G sum_{j in group} m_j R(r_ij) d/r^3,
 * R = prod_{k<L} (1 - K(r; rho_k)) with the levels' current radii, from
 * their state before the drift, integrated by Bulirsch-Stoer extrapolation of
 * the modified midpoint rule (step sequence 2, 4, ..., 16; each step accepted
 * when the last two extrapolations agree within p->bs_eps relative to the
 * state's magnitude, else halved).  Groups of up to 8 bodies take 8 lanes of
 * a wave, groups of up to 512 one workgroup, larger groups all workgroups of
 * one launch together (grid-wide barriers between the force evaluations,
 * Sect. 6.1); a group of more than GENGA_GROUP_MAX bodies sets GENGA_E_GROUP
 * and keeps its drift.
 *
 * Collisions (Sect. 7; b->R non-null, direct = 1): after each accepted
 * Bulirsch-Stoer step the group's first pair (member order) with
 * r < R_i + R_j is traced back to its contact by bisection of that step's
 * length, until the overlap is below p->coll_tol of R_i + R_j, and merged
 * there: the more massive body (the lower index for equal masses) takes
 * x = (m_i x_i + m_j x_j)/(m_i + m_j), v likewise, m_i + m_j and
 * R = (R_i^3 + R_j^3)^(1/3); the other becomes a massless, sizeless ghost at
 * rest at (1e6 + index, 0, 0) (far from every body; the caller may compact
 * the arrays); the lost energy 1/2 m_i m_j/(m_i + m_j)|v_i - v_j|^2
 * - G m_i m_j / r_ij is recorded (genga_collisions).  Spin is not tracked.
 * ws must be sized with the same params (genga_workspace_bytes); every
 * level runs in binary64 on the device, with no host synchronisation, so
 * a step can be captured in a graph.  Not with test-particle modes
 * (GENGA_E_UNSUPPORTED). */
int genga_step(genga_bodies *b, const genga_params *p, genga_pairs *pairs, void *ws, void *stream);

/* Sizes of the symplectic levels' lists in the last genga_step with these
 * params (slevels > 1): out[0] = |E_0| (the true level-0 count) and, for
 * l = 1 .. slevels - 1, the sum of |E_l| over all sub-steps of level l
 * (E_{slevels-1} holds the pairs left to the direct solver).  out is a host
 * array of slevels int64; synchronises the stream. */
int genga_level_counts(int64_t n, const genga_params *p, void *ws, int64_t *out, void *stream);

/* Collisions of the last genga_step with these params (direct = 1, radii
 * given): *count receives their number; up to `cap` records go to the host
 * arrays i (survivor), j (absorbed body) and du (lost energy), sorted by
 * (i, j).  At most 4096 records are kept per step (*count may be larger).
 * Synchronises the stream. */
int genga_collisions(int64_t n, const genga_params *p, void *ws, int64_t *count, int32_t *i,
                     int32_t *j, double *du, int64_t cap, void *stream);

/* Direct solver statistics of the last genga_step with these params (direct
 * = 1): out[0] = groups integrated (summed over the deepest level's
 * sub-steps), out[1] = the largest group's size.  out is a host array of 2
 * int64; synchronises the stream. */
int genga_group_stats(int64_t n, const genga_params *p, void *ws, int64_t *out, void *stream);

/* General relativity (Sect. 3): the post-Newtonian acceleration of every
 * body about the star (eq. apn),
 *   a_i = -mu_i / (r_i^2 c^2) [ -2 (2 - eta_i) rdot_i u_i
 *          + ((1 + 3 eta_i) u_i.u_i - 3/2 eta_i rdot_i^2 - 2 (2 + eta_i) mu_i / r_i) x_i / r_i ],
 * mu_i = G (m_star + m_i), eta_i = m_star m_i / (m_star + m_i)^2, rdot_i =
 * u_i.x_i / r_i, in heliocentric velocities u_i = v_i + P / m_star
 * (P = sum_j m_j v_j), applied over h by the implicit midpoint rule (eq.
 * implicit: u' = u + h a(x, (u + u') / 2), iterated from the explicit guess
 * until the change is below 1e-16 |u'|, at most 50 times); the barycentric
 * velocities are then v'_i = u'_i - P' / m_star with
 * P' = sum_j m_j u'_j / (1 + M / m_star), M = sum_j m_j (total momentum
 * stays zero).  c = p->c_light (> 0).  Momentum sums run in a fixed order.
 * genga_step with c_light > 0 applies it after its first half kick and
 * before its second (a symmetric step); only for the single-system base step
 * (GENGA_E_UNSUPPORTED with levels, the direct solver, test-particle modes,
 * batches). */
int genga_gr_kick(genga_bodies *b, const genga_params *p, double h, void *ws, void *stream);

/* Energy bookkeeping in binary64: the Hamiltonian of the democratic
 * heliocentric splitting (Sect. 2, eqs. H, Ha, Hb, Hc), whose parts the
 * changeover only redistributes (K + (1 - K) = 1), so none of them involves rc:
 *   T   = sum_i m_i |v_i|^2 / 2,
 *   U_* = -G m_star sum_i m_i / |x_i|,
 *   U   = -G sum_{i<j} m_i m_j / r_ij,
 *   C   = |sum_i m_i v_i|^2 / (2 m_star).
 * Writes out[0..4] = (T + U_* + U + C, T, U_*, U, C), `out` a device array
 * of 5 doubles.  Reads x..vz, m.  Asynchronous; two coincident bodies set
 * GENGA_E_NONFINITE in the workspace status.  ws: genga_workspace_bytes(n, p). */
int genga_energy(const genga_bodies *b, const genga_params *p, double *out, void *ws,
                 void *stream);

/* E_K (the force reading of eq. Hb, Sect. 2): the energy whose pair potential
 * is the changeover potential, the one the step without the direct solver
 * conserves for fixed critical radii,
 *   E_K = E + sum_{i<j, r_ij < rho_ij} G m_i m_j [1/r - 1/rho - int_{max(r, 0.1 rho)}^{rho} K(s)/s^2 ds],
 * with rho_ij = max(rc_i, rc_j) from b->rc.  Computes the encounter list of
 * the current positions into `pairs` (as genga_encounter_pairs; device
 * memory, capacity for all of them, else GENGA_E_OVERFLOW in the status and
 * only the first `capacity` pairs count), the integral by the 32-point
 * Gauss-Legendre rule.  Writes out[0..4] as genga_energy and out[5] = E_K
 * (out: device array of 6 doubles).  Asynchronous. */
int genga_energy_k(const genga_bodies *b, const genga_params *p, genga_pairs *pairs, double *out,
                   void *ws, void *stream);

/* ------------------------------------------------------------------------
 * Adjoint (vector-Jacobian products) of the operators above, for gradients of
 * final states with respect to initial conditions and masses.  Each call
 * ACCUMULATES into the caller's adjoint arrays (device, length n each).
 * ------------------------------------------------------------------------ */
typedef struct {
    double *x, *y, *z;    /* adjoints of positions   */
    double *vx, *vy, *vz; /* adjoints of velocities  */
    double *m;            /* adjoints of masses      */
    double *rc;           /* adjoints of r_crit      */
} genga_adjoint;

/* Kick VJP at the positions, masses and radii of b.  With abar = scale * (abx,
 * aby, abz) (the adjoint of the accelerations; scale = h for v += h a):
 *   adj.x  += G sum_j [w u + (w_r / r)(d.u) d],  u = m_k abar_j - m_j abar_k,
 *   adj.m  -= G sum_j w d.abar_j,
 *   adj.rc += G sum_{j: k owns rho} K'(y) d.u / (0.9 rho^2 r^2),
 * with d = x_j - x_k, w = K / r^3, w_r / r = K' / (0.9 rho r^4) - 3 K / r^5 and
 * rho_kj owned by the body with the larger r_crit (ties: the lower index).
 * Same tiling and candidate test as genga_kick; FP64. */
int genga_kick_vjp(const genga_bodies *b, const genga_params *p, double scale,
                   const double *abx, const double *aby, const double *abz, genga_adjoint *adj,
                   void *ws, void *stream);

/* VJP of genga_rcrit at b: reads adj.rc, adds into adj.x.., adj.vx.., adj.m
 * (the branch of the max follows the forward: Hill term on ties). */
int genga_rcrit_vjp(const genga_bodies *b, const genga_params *p, genga_adjoint *adj, void *ws,
                    void *stream);

/* VJP of genga_hc(h) at the velocities and masses of b: with S = sum_i adj.x_i,
 *   adj.v_j += (h m_j / m_star) S,  adj.m_j += (h / m_star) v_j . S;
 * adj.x is unchanged (it passes through). */
int genga_hc_vjp(const genga_bodies *b, const genga_params *p, double h, genga_adjoint *adj,
                 void *ws, void *stream);

/* VJP of genga_drift(dt) taken at the INPUT state of the drift (b): overwrites
 * adj.x.., adj.vx.. (adjoints of the drifted state) with the adjoints of the
 * input state, by reverse mode through the universal-variable solution and
 * implicit differentiation of Kepler's equation. */
int genga_drift_vjp(const genga_bodies *b, const genga_params *p, double dt, genga_adjoint *adj,
                    void *ws, void *stream);

/* ------------------------------------------------------------------------
 * Batched ensembles (the multi-simulation mode named in Sect. 10, not
 * described by the paper): S independent systems, each advanced by the same
 * operators as above, stored back to back in one genga_bodies (n = total).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t S;                /* number of systems, >= 1                              */
    const int64_t *offsets;   /* HOST array of S + 1 body offsets: system s holds
                                 bodies [offsets[s], offsets[s+1]); offsets[0] = 0,
                                 every system non-empty                              */
    const double *m_star;     /* DEVICE arrays of S values: central mass, time step */
    const double *dt;         /*   and the factors n1, n2 of eq. (rcrit) per system  */
    const double *n1;
    const double *n2;
} genga_batch;

/* Workspace size for a batch with these params (0 if the batch is invalid). */
size_t genga_batch_workspace_bytes(const genga_batch *bt, const genga_params *p);

/* Write the batch plan into the workspace: kick tiles (rows of one system
 * against a column range of the same system, sorted by decreasing cost),
 * the body-to-system map and the column slices per system.  Copies from the
 * host and synchronises the stream.  Call once per (batch layout, params,
 * workspace) before the batched calls below; they read the plan. */
int genga_batch_plan(const genga_batch *bt, const genga_params *p, void *ws, void *stream);

/* Shape of the plan: out5 = {tiles, persistent blocks, threads per block,
 * rows per thread, columns per tile} of the one-sided kick.  A binary64 batch
 * without GENGA_FLAG_DIRECTED runs the symmetric kick instead (one block of
 * 256 threads per tile of 512 rows x 512 columns of one system; the plan
 * holds both). */
int genga_batch_info(const genga_batch *bt, const genga_params *p, int64_t *out5);

/* Kick of every system in one persistent launch: for body i of system s,
 * v_i += hfac * dt_s * a_i with a_i summed over the bodies of s only (the
 * formula of genga_kick).  ax/ay/az (nullable) receive a.  pairs (nullable)
 * receives one list for the whole batch with global body indices, in
 * canonical order (which is also system order). */
int genga_kick_batched(const genga_bodies *b, const genga_batch *bt, const genga_params *p,
                       double hfac, double *ax, double *ay, double *az, genga_pairs *pairs,
                       void *ws, void *stream);

/* One base step (as genga_step) of every system with its own m_star, dt, n1,
 * n2; p->G is shared.  The launch sequence is fixed, so the call can be
 * captured in a hipGraph (with GENGA_FLAG_NOSYNC). */
int genga_step_batched(genga_bodies *b, const genga_batch *bt, const genga_params *p,
                       genga_pairs *pairs, void *ws, void *stream);

/* ------------------------------------------------------------------------
 * Self-tuning of launch shapes (GENGA II tunes its kernel parameters at
 * start-up by timing them, Sect. 8).  Candidate shapes are timed with hipEvents
 * (median of 3 after one warm-up) on the caller's own bodies with a zero step
 * factor, so positions and velocities are not modified (the kick's status
 * checks still run).  The fastest shape is written into *p.  With cache_path
 * non-null the choice is first looked up in, and after tuning appended to, a
 * plain-text file: one line "key block ipt tile_cols grid slices ms" per
 * problem, key = kind, device architecture, precision and problem signature
 * (N rounded up to a power of two; or S, total N and a histogram of the system
 * sizes); the last line of a key wins.  ms_out (nullable) receives the time
 * of one kick with the chosen shape (genga_autotune_batched: of a step's two
 * kicks, one without and one with the encounter list).  Synchronises the
 * stream.
 * ------------------------------------------------------------------------ */

/* Workspace for genga_autotune_batched: the largest any candidate needs,
 * then room for the tuner's own encounter list (16 pairs per body). */
size_t genga_autotune_batched_workspace_bytes(const genga_batch *bt, const genga_params *p);

/* Batched kick.  Candidates, in this order: (binary64) the symmetric form
 * with the plan's own slice width (p->slices = 0) and with 1, 2 or 4 column
 * slices per 512-row group, then the one-sided form with block {64, 256} x
 * rows per thread {1, 2} x tile_cols {256, 512, 1024, 2048} x grid {library
 * choice, 32 waves per CU}; each timed 5 times (median) over a kick without
 * and a kick with an encounter list (the list placed after the largest
 * candidate's workspace; both kicks without it if ws_bytes leaves no room),
 * a later candidate chosen only if more than 1 % faster.  Writes p->block, p->ipt,
 * p->tile_cols, p->grid, p->slices and the form flag in p->flags.  On return
 * ws holds the plan of the chosen shape (as after genga_batch_plan).
 * ws_bytes >= genga_autotune_batched_workspace_bytes(bt, p), else candidates
 * that do not fit are skipped.  GENGA_E_UNSUPPORTED if no candidate ran. */
int genga_autotune_batched(const genga_bodies *b, const genga_batch *bt, genga_params *p,
                           void *ws, size_t ws_bytes, const char *cache_path, double *ms_out,
                           void *stream);

/* Workspace for genga_autotune: the largest any candidate needs. */
size_t genga_autotune_workspace_bytes(int64_t n, const genga_params *p);

/* Single-system kick.  Candidates: the one-sided form with rows per thread
 * {1, 2} x column slices {library choice, 8, 16, 32, 64}, and (without a
 * test-particle mode) the symmetric form with slices {library choice, 1, 2, 4,
 * 8} (see genga_params.slices).  Writes p->ipt, p->slices and the form
 * (GENGA_FLAG_DIRECTED or GENGA_FLAG_SYMMETRIC in p->flags, the other form
 * flag cleared).  Cache lines written before the symmetric form existed
 * (seven fields) read as the library's form. */
int genga_autotune(const genga_bodies *b, genga_params *p, void *ws, size_t ws_bytes,
                   const char *cache_path, double *ms_out, void *stream);

/* Symplectic-level configuration (Sect. 6.2: each choice of levels and
 * sub-steps runs for a number of time steps before the simulation, the
 * fastest is kept, and the test is repeated as the system changes).
 * Candidate c is (levels[c], substeps[c]) (host arrays of ncand); each runs
 * one untimed and `steps` timed genga_step calls on the caller's bodies with
 * the other fields of *p, so the state ADVANCES by ncand * (steps + 1) steps,
 * all of them ordinary steps of the integration.  Writes p->slevels and
 * p->substeps of the fastest; ms_out (nullable, host, ncand) receives each
 * candidate's time per step, or -1 where the workspace (ws_bytes) was too
 * small for it or a step reported an error (e.g. GENGA_E_OVERFLOW: raise
 * p->level_capacity).  GENGA_E_UNSUPPORTED if no candidate ran.
 * Synchronises the stream. */
int genga_tune_levels(genga_bodies *b, genga_params *p, const int *levels, const int *substeps,
                      int ncand, int steps, void *ws, size_t ws_bytes, double *ms_out,
                      void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GENGA_H */
