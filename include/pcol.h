/*
 * pcol.h -- deterministic hard-sphere binary collision step on one AMD MI355X
 * (gfx950).  C ABI over hand-written HIP kernels.
 *
 * The operation is the hard-sphere collision operator of Schwarz, Kopper,
 * de Staercke and Beck, "Efficient computation of particle-fluid and
 * particle-particle interactions in compressible flow" (arXiv 2501.05340):
 *
 *   - Sec. "Particle Collisions", eq. (detect1/detect2): within a step of
 *     length dt two spheres moving on straight lines collide at the lower of
 *     the two positive roots t of |dx + t dv|^2 = (r_i + r_j)^2 if it is <= dt
 *     and the spheres approach each other.
 *   - Sec. "Inter-Particle Collisions": momentum jump relations with the normal
 *     impulse J_n = -m_r (1 + e) (v_r . n_p), v_r = v_1 - v_2, n_p the unit
 *     vector from sphere 1 to sphere 2, m_r = m_1 m_2 / (m_1 + m_2); friction
 *     coefficient 0 (no tangential impulse, no spin) except in pcol_step_spin,
 *     which adds the tangential impulse and the spin update.
 *   - eq. (update_vel1/update_vel2/update_rho): new velocities v + J/m, and the
 *     sphere is moved to the contact point and flies the rest of the step with
 *     its new velocity.
 *   - Sec. "Collision Operator": one collision per sphere per step; spheres
 *     that collided leave the set of eligible partners.
 *   - Sec. "Intersection of Particles with Solid Walls" (pcol_step_walls only):
 *     reflective walls on chosen axes.
 *   - Sec. "Dispersed Phase" and Sec. "Deposition" (pcol_deposit only): the
 *     linear projection of per-particle sources onto element corner nodes.
 *
 * THE ORDERING RULE (the paper asks only for a deterministic order; this is
 * the order-independent rule every entry point computes):
 *   1. The contact time of an active pair (i, j) is computed in IEEE-754
 *      binary64, round to nearest, without FMA contraction, in exactly this
 *      order:  d_k = x_j,k - x_i,k, then if d_k > L_k/2: d_k -= L_k, else if
 *      d_k < -L_k/2: d_k += L_k;  u_k = v_j,k - v_i,k;  s = r_i + r_j;
 *      a = (u0 u0 + u1 u1) + u2 u2;  b = (d0 u0 + d1 u1) + d2 u2;
 *      c = ((d0 d0 + d1 d1) + d2 d2) - s s;  a collision exists iff
 *      a > 0, b < 0, c > 0 and D = b b - a c >= 0; then t = c / (-b + sqrt(D))
 *      and the collision is kept iff t <= dt.  (t_ij == t_ji bitwise.)
 *   2. partner(i) = the active j != i minimising (t_ij, j) lexicographically:
 *      exact binary64 comparison of t, exact ties to the smaller caller index.
 *   3. A sweep resolves every pair with partner(i) = j and partner(j) = i, all
 *      at once, using start-of-step positions and velocities, and removes both
 *      spheres from the active set.  Sweeps repeat until one finds no mutual
 *      pair (the globally earliest pair is always mutual, so each sweep with a
 *      remaining contact resolves at least one pair).
 *   4. Resolve of i with partner j at time t (same d, u, s as in 1):
 *      n_k = (d_k + t u_k) / s;  g = (u0 n0 + u1 n1) + u2 n2;
 *      m_r = (m_i m_j) / (m_i + m_j);  J = (m_r (1 + e)) g;
 *      v_i,k' = v_i,k + (J / m_i) n_k;  x_i,k' = (x_i,k + t v_i,k) + (dt - t) v_i,k'.
 *      (For j the same with the roles swapped; the result is bitwise
 *      independent of which sphere is called i.)
 *   5. Spheres without a collision: x' = x + dt v.  Every final coordinate is
 *      wrapped: if x' >= L: x' -= L, else if x' < 0: x' += L; a result equal to
 *      L becomes 0.
 *
 * Data: structure-of-arrays, binary64, N <= 2^31 - 1 spheres.  All array
 * pointers are DEVICE pointers owned by the caller; the library owns only the
 * scratch inside pcol_ctx.  Calls enqueue work on the context's HIP stream.
 * Entry points that validate data on the device read back a few bytes and so
 * synchronise with that stream; they say so below.  Errors in arguments or
 * data are reported before any kernel writes caller memory (caller arrays are
 * then unchanged), except PCOL_E_SWEEPS, see pcol_step.  No C++ exception
 * crosses this interface.
 */
#ifndef PCOL_H
#define PCOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcol_ctx pcol_ctx;

typedef enum {
  PCOL_OK = 0,
  PCOL_E_INVALID = 1, /* bad argument, or data that is non-finite, r <= 0, m <= 0, or a
                         position outside [0, L) */
  PCOL_E_BOX = 2,     /* some box side L_k <= 2 * reach, reach = 2 max r + 2 max|v| dt:
                         the minimum image would no longer be unique */
  PCOL_E_NOMEM = 3,   /* device allocation failed */
  PCOL_E_HIP = 4,     /* a HIP runtime call failed; see pcol_last_error */
  PCOL_E_SWEEPS = 5,  /* opts.max_sweeps sweeps ran and the last still resolved pairs */
  PCOL_E_STATE = 6,   /* call order: pcol_detect / pcol_resolve before pcol_bin, or for a
                         different particle count than the last pcol_bin */
  PCOL_E_SCRATCH = 7  /* pcol_deposit_noalloc: the input needs more than the library's
                         fixed device scratch (PCOL_NOALLOC_SCRATCH_BYTES) */
} pcol_status;

/* The spheres.  x, y, z in [0, len_k); r > 0 (radius: the paper's diameter is 2r);
 * m > 0.  Positions and velocities are updated in place by pcol_resolve,
 * pcol_advance and pcol_step. */
typedef struct {
  int64_t n;
  double *x, *y, *z;
  double *vx, *vy, *vz;
  const double *r;
  const double *m;
} pcol_particles;

/* periodic box [0, len0) x [0, len1) x [0, len2) */
typedef struct {
  double len[3];
} pcol_box;

typedef struct {
  double cell_mult;   /* grid cell side >= reach * cell_mult, cell_mult >= 1 (default 1) */
  int max_sweeps;     /* 0: no cap (a step needs at most n/2 + 1 sweeps); pcol_step_batched:
                         sweeps captured in its graph (see there) */
  int home_cells;     /* consecutive home cells per workgroup of the sweep-1 pair test, whose
                         filter survivors are decided together (0: automatic, 4 when the
                         cells average under 24 spheres, else 1; at most 16).  Results do
                         not depend on it. */
  int contact_slots;  /* contacts kept per sphere from the sweep-1 detect; spheres with more
                         fall back to an exact neighbourhood search (default 12) */
  int filter;         /* pair filter ahead of the exact rule (same results for every value):
                         0 binary64 filter in Gram form; 1 binary32 filter, contact distance
                         inflated by a band, survivors decided in binary64. */
  double band_rel;    /* FP32 filter safety band, relative to r_i + r_j (default 1e-4) */
  int timing;         /* 1: time kernels with HIP events; times land in pcol_stats */
  int autotune;       /* pcol_step_batched: 1 = pick cell size and home cells per workgroup
                         by timing candidates on the first call (cached, see
                         pcol_step_batched); 0 = opts.cell_mult and 4 cells */
  double split_quantile; /* extent split (default 0.999; 0 or 1 = off): the spheres whose extent
                         r + |v| dt lies above this quantile are searched separately, so the
                         grid's cells need only twice the quantile extent instead of the reach.
                         Used when that shrinks the cells by 15% or more.  Results do not
                         depend on it. */
  int order;          /* which pairs collide (pcol_step only; pcol_detect, pcol_resolve and
                         the other steps always use rule 2):
                         0: rules 2-3 (each sphere's earliest partner, mutual pairs per sweep);
                         1: the order of Sec. "Collision Operator" taken literally: elements
                         along a space-filling curve, the particles of an element one after
                         another, each still eligible particle taking the first eligible
                         partner with a contact (rule 1) found in its candidate elements in
                         curve order, both then leaving the eligible set.  The elements are
                         the cells of the curve grid, cell side >= reach = 2 max r +
                         2 max|v| dt (floor(L_k / (reach (1 + 1e-9))) cells per axis, between
                         1 and 2048), a sphere's cell floor(x_k / h_k) (h_k = L_k / cells,
                         clamped to the last cell); the curve is the Morton order (bits of
                         the cell coordinates interleaved, x lowest); particles of a cell in
                         caller-index order.  With rank(i) = (Morton code of i's cell,
                         caller index), that pass is the greedy matching of the contact graph
                         taking edges by (lower rank of the two ends, higher rank), computed
                         here in parallel: every active sphere points at its active contact
                         of smallest rank, mutual pairs collide (rule 4) and leave, sweep
                         after sweep.  Default 0. */
} pcol_opts;

typedef struct {
  int64_t n_pairs;       /* collisions resolved */
  int64_t n_sweeps;      /* sweeps run, including the last one that resolved nothing */
  int64_t pair_tests;    /* unordered candidate pairs tested geometrically (the half stencil
                            plus the separate search of the spheres above the split extent) */
  int64_t contacts;      /* unordered pairs with a contact within dt (sweep 1) */
  int64_t n_overflow;    /* spheres whose contacts exceeded contact_slots */
  int64_t n_recheck;     /* survivors of filter 1 decided by the binary64 rule */
  int32_t nc[3];         /* grid cells per axis */
  int32_t home_cells;    /* home cells per workgroup of the sweep-1 pair test (0: the exact
                            per-sphere search of a box with fewer than 3 cells on an axis) */
  int32_t max_cell;      /* largest cell occupancy */
  double h[3];           /* grid cell side per axis */
  double reach;          /* 2 max r + 2 max|v| dt */
  double band;           /* FP32 filter band in use (>= band_rel; 0 without the filter) */
  double ms_bin;         /* with opts.timing only: validation, reach, binning */
  double ms_detect;      /*   the sweep-1 pair-test kernel alone */
  double ms_sweeps;      /*   partner selection and all resolve sweeps */
  double ms_advance;     /*   free flight and wrap */
  int64_t n_wide;        /* spheres above the split extent (searched separately; 0 = no split) */
  double rho_c;          /* split extent in use (0 = no split) */
} pcol_stats;

/* Fill *opts with the defaults listed above. */
void pcol_default_opts(pcol_opts *opts);

/* Create a context for up to n_max spheres on the current HIP device.
 * hip_stream: a hipStream_t (NULL = the default stream).  opts: nullable.
 * Allocates O(n_max) device scratch; returns PCOL_E_NOMEM if that fails. */
pcol_status pcol_create(pcol_ctx **out, int64_t n_max, void *hip_stream, const pcol_opts *opts);

/* Release the context and its device scratch (NULL is ignored). */
void pcol_destroy(pcol_ctx *ctx);

/* Text of the last error reported on this context (never NULL). */
const char *pcol_last_error(const pcol_ctx *ctx);

/* Change the stream later calls enqueue on. */
pcol_status pcol_set_stream(pcol_ctx *ctx, void *hip_stream);

/* Bin the spheres (Sec. "Collision Operator": particles are sorted by host
 * cell and counted per cell): validates the data, computes
 * reach = 2 max r + 2 max|v| dt and a uniform grid of cell side >= reach *
 * cell_mult per axis, and keeps a cell-sorted copy of the start-of-step state
 * in the context.  Reads only.  Synchronises (reads back the reach and the
 * largest cell).  A call with the sphere count, box, dt and walls of the
 * context's last binning counts the spheres into that binning's grid during
 * the reach pass and keeps those counts when this call's reach gives the same
 * grid (the grid is always the one this call's reach determines). */
pcol_status pcol_bin(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt);

/* Earliest partner of every active sphere over the active set (rule 1-2),
 * from the state kept by the last pcol_bin (p must be the binned set).
 * active: device uint8[n], nonzero = active; NULL = all active.
 * key_out: device uint64[n]:  (bits of (float)t_min) << 32 | partner index,
 *          or UINT64_MAX when no active sphere collides with i (or i inactive).
 * tmin_out: device double[n] (nullable): the exact binary64 t_min, +inf if none.
 * Indices are caller indices.  Asynchronous. */
pcol_status pcol_detect(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt,
                        const uint8_t *active, uint64_t *key_out, double *tmin_out);

/* One sweep of rule 3-4 from keys made by pcol_detect: for every active i whose
 * partner j has i as its partner, sphere i gets its post-collision velocity and
 * end-of-step position (written into p), active[i] = 0, partner[i] = j,
 * tcoll[i] = t.  Start-of-step data come from the last pcol_bin, so p may
 * already hold results of earlier sweeps.  n_pairs_dev: device int64 scalar,
 * incremented by the number of pairs resolved (nullable).  Spheres not in a
 * mutual pair are untouched.  Asynchronous. */
pcol_status pcol_resolve(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                         double e, const uint64_t *key, uint8_t *active, int32_t *partner,
                         double *tcoll, int64_t *n_pairs_dev);

/* Free flight (rule 5) of every sphere with partner[i] < 0, in place, from the
 * positions and velocities currently in p.  Asynchronous. */
pcol_status pcol_advance(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                         const int32_t *partner);

/* The whole step (rules 1-5): bin, sweeps until none resolves a pair, free
 * flight and wrap; p is updated in place.  partner (device int32[n], nullable):
 * the caller index of the sphere i collided with, or -1.  tcoll (device
 * double[n], nullable): contact time within the step, NaN if none.
 * stats (host, nullable).  Synchronises once after validation, once after sweep
 * 1 (and after binning for the binary32 filter), then once per sweep for a
 * short sweep list, or once per group of sweeps run on the device for a long
 * one.  On PCOL_E_SWEEPS p is left as it was (the end-of-step state is written
 * only once the sweeps are done). */
pcol_status pcol_step(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt, double e,
                      int32_t *partner, double *tcoll, pcol_stats *stats);

/* pcol_step with angular velocities and Coulomb friction (Sec. "Inter-Particle
 * Collisions": the impulse J = J_n n_p + J_t t_p with
 * J_t = max(mu J_n, -(2/7)(1+e) m_r |v_rt|), sliding or sticking, t_p along the
 * tangential contact-point velocity v_rt; the jump relations of momentum and
 * angular momentum, with the moment of inertia of a solid sphere
 * I = m d^2 / 10, Sec. "Dispersed Phase").
 * wx, wy, wz: device double[n] angular velocities in the caller's order, read at
 * the start of the step and updated in place for the spheres that collide
 * (the others keep theirs); validated with the other inputs (non-finite:
 * PCOL_E_INVALID, nothing changed).  mu: friction coefficient, >= 0.
 * Contact times do not depend on the spins, so the pair set is pcol_step's;
 * with mu = 0 every output equals pcol_step's bitwise and the spins are
 * unchanged.  Everything else as pcol_step (on PCOL_E_SWEEPS the spins of the
 * pairs resolved so far have been updated, p has not). */
pcol_status pcol_step_spin(pcol_ctx *ctx, pcol_particles *p, double *wx, double *wy, double *wz,
                           const pcol_box *box, double dt, double e, double mu,
                           int32_t *partner, double *tcoll, pcol_stats *stats);

/* Statistics of one pcol_step_batched call. */
typedef struct {
  int64_t n_pairs;       /* collisions resolved over all boxes */
  int64_t n_sweeps;      /* sweeps of the step (the slowest box decides) */
  int64_t contacts;      /* unordered pairs with a contact within dt */
  int64_t n_overflow;    /* spheres whose contacts exceeded contact_slots, summed over sweeps */
  int64_t total_cells;   /* cells of all boxes */
  int32_t replanned;     /* 1 if this call (re)built the per-box grids and the graph */
  int32_t finished_on_host; /* 1 if the captured sweeps did not suffice and the host finished */
  int32_t tuned;         /* 1 if this call ran the autotuner */
  int32_t home_cells;    /* chosen home cells per workgroup of the pair-test launch */
  double cell_mult;      /* chosen cell size factor */
} pcol_batch_stats;

/* Step many independent periodic boxes at once (the batched form).  Box b owns
 * spheres [box_off[b], box_off[b+1]) of the concatenated arrays in p and the
 * periodic box boxes[b]; every box follows rules 1-5 on its own (spheres of
 * different boxes never interact).  box_off (nbox + 1 entries, box_off[0] = 0,
 * box_off[nbox] = p->n) and boxes are HOST arrays.
 *
 * Each box gets its own grid (cell side >= the box's reach times cell_mult,
 * at least 3 cells per axis: a box with L_k < 3 reach is rejected with
 * PCOL_E_BOX).  The whole step (validation, binning, one persistent pair-test
 * launch over the cells of all boxes, up to a planned number of sweeps with a
 * device flag ending them early, free flight) is captured once into a HIP
 * graph and replayed by later calls with the same arrays, layout, dt and e.
 * The graph re-validates on the device each step: if a box's reach has
 * outgrown its planned cells, the host re-plans and re-captures before any
 * state changes; if the planned sweeps do not finish the step, the host runs
 * the remaining sweeps.  Results equal pcol_step applied box by box: partner
 * holds global indices (sphere k of box b is box_off[b] + k), which order the
 * spheres of a box as their local indices do, so rule 2's ties break alike.
 * Every step runs to completion: opts.max_sweeps > 0 fixes the number of
 * sweeps captured in the graph (the host runs any beyond them); with 0 the
 * graph starts with 12 and is re-captured with more after a step that needed
 * more.
 * With opts.autotune, the first call times candidate cell sizes and home cells
 * per workgroup on scratch copies of the input and keeps the fastest; choices are
 * cached in the text file named by the environment variable PCOL_TUNE_CACHE
 * (default $HOME/.cache/pcol_tune.txt), keyed by GPU and batch shape.
 * Synchronises once per call (plus planning and tuning calls). */
pcol_status pcol_step_batched(pcol_ctx *ctx, int32_t nbox, const int64_t *box_off,
                              const pcol_box *boxes, pcol_particles *p, double dt, double e,
                              int32_t *partner, double *tcoll, pcol_batch_stats *stats);

/* Gradient of a scalar loss with respect to the positions and velocities of
 * all spheres (device arrays, caller order, n each). */
typedef struct {
  double *x, *y, *z;
  double *vx, *vy, *vz;
} pcol_state_grad;

/* One pcol_step with reflective walls at 0 and len_k on every axis k with
 * walls[k] != 0 (host array of 3; the other axes stay periodic): Sec.
 * "Intersection of Particles with Solid Walls" with a perfectly reflective wall,
 * and the condition of Sec. "Particle Collisions" that a collision must occur
 * before an intersection with a domain boundary.  The particle is tracked by its
 * centre.  Rules 1-5 change as follows:
 *   1. along a wall axis d_k = x_j,k - x_i,k (no minimum image), and a contact
 *      at t is kept only if t <= T_i and t <= T_j, where T is the centre's time
 *      of flight to a wall plane: the least over wall axes with v_k != 0 of
 *      (len_k - x_k) / v_k for v_k > 0 and -x_k / v_k for v_k < 0 (+inf if none);
 *   4, 5. a final coordinate p (free flight, or the rest of the step after a
 *      collision) along a wall axis is reflected: p >= len: p = len - (p - len),
 *      p < 0: p = -p, and the velocity component changes sign; a result equal
 *      to len becomes the largest double below len.
 * Positions stay in [0, len_k).  Every filter form works with walls; pcol_bin,
 * pcol_detect and pcol_resolve do not (pcol_detect and pcol_resolve after this
 * call return PCOL_E_STATE until pcol_bin runs again).  Otherwise as pcol_step. */
pcol_status pcol_step_walls(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box,
                            const int32_t walls[3], double dt, double e, int32_t *partner,
                            double *tcoll, pcol_stats *stats);

/* pcol_step_spin between reflective walls (walls as in pcol_step_walls): the
 * friction resolve of pcol_step_spin with the separation and flight of
 * pcol_step_walls.  An elastic wall changes no spin (its momentum change is
 * zero, so the angular jump relation of Sec. "Intersection of Particles with
 * Solid Walls" gives none).  Arguments, errors and synchronisation as
 * pcol_step_spin. */
pcol_status pcol_step_spin_walls(pcol_ctx *ctx, pcol_particles *p, double *wx, double *wy,
                                 double *wz, const pcol_box *box, const int32_t walls[3],
                                 double dt, double e, double mu, int32_t *partner, double *tcoll,
                                 pcol_stats *stats);

/* Adjoint of one pcol_step with its pair set held fixed (reverse mode; the
 * derivative of rule 4 and of the contact time of rule 1, which depends on the
 * start positions and velocities through |d + t u| = r_i + r_j).  For a
 * multi-step rollout call it once per step in reverse order; the checkpoint of
 * a step is its start state and its pair record.
 *   start:   the step's start-of-step state (x, y, z, vx, vy, vz, r, m), read only.
 *   partner, tcoll: that step's outputs of pcol_step (device, caller order).
 *   g_out:   gradient with respect to the step's end-of-step state (read only).
 *   g_in:    receives the gradient with respect to the start state; its arrays
 *            must not alias g_out's.
 *   ge:      device double scalar; the gradient with respect to e is ADDED to it
 *            (summed in a fixed order, so repeated runs agree bitwise).
 * Positions are differentiated through the periodic wrap as the identity (the
 * wrap shifts by a constant).  Uses context scratch for n_max spheres; no
 * readback, asynchronous. */
pcol_status pcol_step_backward(pcol_ctx *ctx, const pcol_particles *start, const pcol_box *box,
                               double dt, double e, const int32_t *partner, const double *tcoll,
                               const pcol_state_grad *g_out, pcol_state_grad *g_in, double *ge);

/* Deposition of per-sphere sources onto the corner nodes of a periodic
 * Cartesian grid: the projection operator of Sec. "Dispersed Phase" (a linear,
 * C0-continuous inverse-distance weighting onto the eight corner nodes of the
 * host element) with the deposition radius equal to the cell size, as in Sec.
 * "Deposition", and the node-wise sum over all spheres.  On cells of equal
 * volume the weights are trilinear:
 *   h_d = L_d / nc_d;  s_d = p_d / h_d;  c_d = min(floor(s_d), nc_d - 1);
 *   f_d = s_d - c_d;  corner b in {0, 1}^3 (b_0 fastest) receives
 *   w = ((b_0 ? f_0 : 1 - f_0) (b_1 ? f_1 : 1 - f_1)) (b_2 ? f_2 : 1 - f_2)
 *   times each component, at node ((c_2 + b_2) mod nc_2, (c_1 + b_1) mod nc_1,
 *   (c_0 + b_0) mod nc_0), node (i, j, k) sitting at (i h_0, j h_1, k h_2).
 * The weights of one sphere sum to 1 (the deposition is conservative) and the
 * operator is the transpose of trilinear interpolation of a node field.
 *   x, y, z: device, n positions, each in [0, L_d) and finite.
 *   a:       device, comp x n sources, a[q * n + i] (1 <= comp <= 8; the paper
 *            carries 4: three momentum components and the energy, each with
 *            the sign the caller wants deposited).
 *   nc, len: host, cells per axis (1 .. 2^20, at most 2^31 - 1 elements in all)
 *            and box sides (> 0).
 *   out:     device, nc_0 nc_1 nc_2 comp doubles, node-major:
 *            out[((k nc_1 + j) nc_0 + i) comp + q]; overwritten.
 * The weights are bitwise those of the formulas above.  The node sums are
 * formed without floating-point atomics: the spheres are counted and scattered
 * by element (a counting sort), each element sums w a over its spheres in
 * caller-index order (scatter order for an element of more than 64 spheres),
 * and each node adds the corner sums of its eight elements in the order
 * b = 0..7.  Repeated calls on the same input therefore agree bit for bit (up
 * to 64 spheres per element); against a sum in caller-index order each node is
 * within 2 (k - 1) 2^-53 sum|w a| (k its number of terms), and a node with one
 * term is exact.  Positions are checked on the device first (one readback, so
 * the call synchronises with the stream); on PCOL_E_INVALID out is unchanged.
 * n = 0 gives zeros.  Scratch: 8 + 16 ceil((4 + comp) / 2) bytes per sphere
 * (72 for comp = 4) and 8 bytes per element, held by the context and grown on
 * demand (independent of n_max); growing it synchronises with the stream. */
pcol_status pcol_deposit(pcol_ctx *ctx, const double *x, const double *y, const double *z,
                         int64_t n, const double *a, int comp, const int32_t nc[3],
                         const double len[3], double *out);

/* Size of the fixed device scratch of pcol_deposit_noalloc (per GPU). */
#define PCOL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* pcol_deposit for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same operation, kernels and results (bitwise equal to pcol_deposit on the
 * same input, up to the order of more than 64 spheres in one element), without
 * a context and without any allocation: no hipMalloc, hipFree, pinned host
 * memory or other allocating call.  Its scratch is a fixed array of
 * PCOL_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, which the library
 * holds from the first call on that GPU until the process ends.  The input must
 * fit: with R = 16 ceil((4 + comp) / 2) bytes per record and ne = nc_0 nc_1
 * nc_2 elements, each rounded up to 256 B, the scratch holds 4n + 4n + Rn +
 * 4(ne + 1) + 4(ne + 1) + 4(ne / 4096 + 2) + 8,232 + 4 bytes (about 72n + 8ne
 * for comp = 4: for example 500k spheres on 3M elements); a larger input
 * returns PCOL_E_SCRATCH before any work, out unchanged.
 *   hip_stream: the hipStream_t to enqueue on (NULL: the default stream) on the
 *   current device.  Other arguments, checks and errors as pcol_deposit; the
 *   position check is read back into host memory, so the call synchronises with
 *   the stream.  Every call on one GPU uses that GPU's one scratch array (the
 *   counts it needs zeroed are cleared by each call): calls that overlap in time
 *   on one GPU, from several threads or on several streams, race and must not
 *   be made.  Returns PCOL_OK, PCOL_E_INVALID, PCOL_E_SCRATCH or PCOL_E_HIP. */
pcol_status pcol_deposit_noalloc(const double *x, const double *y, const double *z, int64_t n,
                                 const double *a, int comp, const int32_t nc[3],
                                 const double len[3], double *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PCOL_H */
