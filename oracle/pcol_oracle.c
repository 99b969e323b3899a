/*
 * pcol oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU statement of one deterministic hard-sphere
 * collision step, written from the paper (Schwarz, Kopper, de Staercke, Beck,
 * "Efficient computation of particle-fluid and particle-particle interactions
 * in compressible flow", arXiv 2501.05340).  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may call it; the GPU library never does,
 * and the two share no code.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off (no fast-math: every
 * floating-point operation below is one IEEE-754 binary64 operation, rounded
 * to nearest, in the order written).
 *
 * What is computed (one step of length dt, periodic box [0,L0)x[0,L1)x[0,L2)):
 *
 *  pair time   Sec. "Particle Collisions", eq. (detect1/detect2): two spheres
 *              moving on straight lines touch when |dx + t dv|^2 = (r_i+r_j)^2.
 *              A collision exists when the quadratic has two positive roots,
 *              the lower one is <= dt, and the spheres approach each other.
 *              orc_pair_time() spells out the operation order used.
 *  earliest    each active sphere's partner is the active sphere with the
 *              smallest contact time, exact ties going to the smaller index
 *              (the paper only asks for a deterministic order; this is the
 *              order-free rule that a parallel sweep can reproduce).
 *  sweeps      Sec. "Collision Operator": one collision per sphere per step;
 *              spheres that collided leave the eligible set.  Every sweep
 *              resolves all mutual earliest pairs at once, removes them, and
 *              recomputes partners over the rest from start-of-step data,
 *              until a sweep finds no mutual pair.
 *  resolve     Sec. "Inter-Particle Collisions", momentum jump relations with
 *              the normal impulse J_n = -m_r (1+e) (v_r . n_p), friction
 *              coefficient 0 (no tangential impulse, no spin), followed by
 *              eq. (update_vel1/update_vel2) and eq. (update_rho): move to the
 *              contact point, then fly the rest of the step with the new
 *              velocity.
 *  free flight spheres without a collision move x + dt v; every position is
 *              wrapped back into [0, L).
 *  deposition  orc_deposit: Sec. "Dispersed Phase" and Sec. "Deposition": a
 *              per-sphere quantity projected linearly onto the eight corner
 *              nodes of the host cell of a periodic Cartesian grid (the
 *              C0-continuous inverse-distance weighting with deposition radius
 *              equal to the cell size, on cells of equal volume: trilinear
 *              weights), summed over all spheres.
 *  literal     orc_step_sequential: the order of Sec. "Collision Operator" and
 *  order       Sec. "Particle-Particle Collisions" taken literally: elements visited
 *              one after another along a space-filling curve, each particle
 *              scanning its candidate elements in curve order and taking the
 *              first valid collision it finds; both particles then leave the
 *              eligible set.  Sequential by definition; it serves to measure
 *              how far the order-free rule above departs from it.
 *  walls       orc_step_walls: the same step with reflective walls on chosen
 *              axes (Sec. "Intersection of Particles with Solid Walls", Sec.
 *              "Particle Collisions"): no minimum image across a wall, a
 *              collision counts only before either sphere's next boundary
 *              intersection, and a centre that reaches a wall plane within the
 *              step is reflected (elastic wall).
 *  friction    orc_step_spin: the same step with angular velocities and
 *              Coulomb friction (coefficient mu) in the resolve: the impulse
 *              gains the tangential part J_t t_p of Sec. "Inter-Particle
 *              Collisions" (sliding or sticking) and the spins change by the
 *              angular jump relations, with the moment of inertia of a solid
 *              sphere from Sec. "Dispersed Phase".
 *
 * Every function below cites the passage it follows.  Pins: tests/test_oracle_*.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FP_CONTRACT OFF

enum {
  ORC_OK = 0,
  ORC_E_INVALID = 1, /* bad argument or non-finite / non-positive data */
  ORC_E_BOX = 2,     /* box side <= 2 * reach on some axis */
  ORC_E_NOMEM = 3,
  ORC_E_SWEEPS = 5   /* sweep cap reached with mutual pairs still found */
};

/* threads the parallel loops below run on (reported beside timings) */
int orc_max_threads(void) { return omp_get_max_threads(); }

/* minimum-image component: the separation along one periodic axis is mapped
 * into [-L/2, L/2] by one subtraction or addition of L */
static double orc_wrap_sep(double d, double len) {
  if (d > 0.5 * len) {
    d = d - len;
  } else if (d < -0.5 * len) {
    d = d + len;
  }
  return d;
}

/*
 * Contact time of spheres i and j within [0, dt], Sec. "Particle Collisions",
 * eq. (detect1/detect2).  With d = x_j - x_i (minimum image) and u = v_j - v_i
 * the contact condition |d + t u|^2 = s^2, s = r_i + r_j, is the quadratic
 *     a t^2 + 2 b t + c = 0,  a = u.u,  b = d.u,  c = d.d - s^2.
 * Two positive roots exist iff a > 0, b < 0 (the spheres approach), c > 0
 * (they are apart now) and D = b^2 - a c >= 0 (a tangent contact counts: "at
 * least one solution").  The lower root is evaluated in the cancellation-free
 * form t = c / (-b + sqrt(D)); the collision is kept iff t <= dt.
 * Sums are accumulated left to right: ((p0 + p1) + p2).
 * Returns 1 and stores t on a collision, else 0.
 */
int orc_pair_time(const double xi[3], const double vi[3], double ri, const double xj[3],
                  const double vj[3], double rj, const double L[3], double dt, double *t_out) {
  double d[3], u[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = orc_wrap_sep(xj[k] - xi[k], L[k]);
    u[k] = vj[k] - vi[k];
  }
  const double s = ri + rj;
  const double a = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
  const double b = (d[0] * u[0] + d[1] * u[1]) + d[2] * u[2];
  const double c = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) - s * s;
  if (!(a > 0.0) || !(b < 0.0) || !(c > 0.0)) return 0;
  const double D = b * b - a * c;
  if (!(D >= 0.0)) return 0;
  const double t = c / (-b + sqrt(D));
  if (!(t <= dt)) return 0;
  *t_out = t;
  return 1;
}

/* the lexicographic order on (t, index) used to pick the earliest partner */
static int orc_before(double t1, int64_t j1, double t2, int64_t j2) {
  return t1 < t2 || (t1 == t2 && j1 < j2);
}

/* reach = 2 r_max + 2 |v|_max dt: the largest centre distance at step start of
 * any pair that can touch within dt (Sec. "Collision Operator": the halo grows
 * with the distance the fastest particle travels; both spheres move) */
static double orc_reach(int64_t n, const double *vx, const double *vy, const double *vz,
                        const double *r, double dt) {
  double v2 = 0.0, rm = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double w = (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
    if (w > v2) v2 = w;
    if (r[i] > rm) rm = r[i];
  }
  return 2.0 * rm + 2.0 * sqrt(v2) * dt;
}

/* a plain uniform cell grid with cell side >= reach * cell_mult (Sec. "Collision
 * Operator": particles are bucketed by host element, and only elements within the
 * halo distance hold candidates).  Besides the particle indices bucketed by cell
 * it keeps a copy of each particle's position, velocity and radius at its
 * bucketed slot (sd[7 k .. 7 k + 6] for item[k]), so that the candidates of a cell
 * are read from consecutive memory; the values are the caller's, unchanged. */
typedef struct {
  int nc[3];
  double h[3];
  int64_t *start; /* ncell + 1 */
  int64_t *item;  /* particle indices bucketed by cell */
  double *sd;     /* x, y, z, vx, vy, vz, r of item[k] at sd + 7 k */
  int nb[3];      /* number of distinct neighbour offsets per axis */
  int off[3][3];  /* the distinct offsets */
} orc_grid;

static int orc_cell_of(double x, double h, int nc) {
  int c = (int)floor(x / h);
  if (c < 0) c = 0;
  if (c > nc - 1) c = nc - 1;
  return c;
}

static int orc_grid_build(orc_grid *G, int64_t n, const double *x, const double *y,
                          const double *z, const double *vx, const double *vy, const double *vz,
                          const double *r, const double L[3], double cell) {
  const double *p[3] = {x, y, z};
  for (int a = 0; a < 3; ++a) {
    int nc = (int)floor(L[a] / (cell * (1.0 + 1e-9)));
    if (nc < 1) nc = 1;
    if (nc > 2048) nc = 2048;
    G->nc[a] = nc;
    G->h[a] = L[a] / nc;
    /* distinct cells among c-1, c, c+1 (periodic); fewer than three cells
     * per axis would otherwise visit a cell twice */
    if (nc >= 3) {
      G->nb[a] = 3;
      G->off[a][0] = -1;
      G->off[a][1] = 0;
      G->off[a][2] = 1;
    } else if (nc == 2) {
      G->nb[a] = 2;
      G->off[a][0] = 0;
      G->off[a][1] = 1;
    } else {
      G->nb[a] = 1;
      G->off[a][0] = 0;
    }
  }
  const int64_t ncell = (int64_t)G->nc[0] * G->nc[1] * G->nc[2];
  G->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  G->item = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *cid = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!G->start || !G->item || !cid) {
    free(G->start);
    free(G->item);
    free(cid);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = orc_cell_of(p[a][i], G->h[a], G->nc[a]);
    cid[i] = ((int64_t)c[2] * G->nc[1] + c[1]) * G->nc[0] + c[0];
    G->start[cid[i] + 1] += 1;
  }
  for (int64_t k = 0; k < ncell; ++k) G->start[k + 1] += G->start[k];
  int64_t *fill = (int64_t *)malloc((size_t)(ncell > 0 ? ncell : 1) * sizeof(int64_t));
  if (!fill) {
    free(G->start);
    free(G->item);
    free(cid);
    return ORC_E_NOMEM;
  }
  memcpy(fill, G->start, (size_t)ncell * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) G->item[fill[cid[i]]++] = i;
  free(fill);
  free(cid);
  G->sd = (double *)malloc((size_t)(n > 0 ? n : 1) * 7 * sizeof(double));
  if (!G->sd) {
    free(G->start);
    free(G->item);
    return ORC_E_NOMEM;
  }
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = G->item[k];
    double *d = G->sd + 7 * k;
    d[0] = x[i];
    d[1] = y[i];
    d[2] = z[i];
    d[3] = vx[i];
    d[4] = vy[i];
    d[5] = vz[i];
    d[6] = r[i];
  }
  return ORC_OK;
}

static void orc_grid_free(orc_grid *G) {
  free(G->start);
  free(G->item);
  free(G->sd);
}

/* cell number q of the neighbour (a0, a1, a2) of cell (c0, c1, c2), periodic */
static int64_t orc_neighbour(const orc_grid *G, int c0, int c1, int c2, int a0, int a1, int a2) {
  const int q0 = (c0 + G->off[0][a0] + G->nc[0]) % G->nc[0];
  const int q1 = (c1 + G->off[1][a1] + G->nc[1]) % G->nc[1];
  const int q2 = (c2 + G->off[2][a2] + G->nc[2]) % G->nc[2];
  return ((int64_t)q2 * G->nc[1] + q1) * G->nc[0] + q0;
}

static int orc_check_inputs(int64_t n, const double *x, const double *y, const double *z,
                            const double *vx, const double *vy, const double *vz,
                            const double *r, const double *m, const double L[3], double dt) {
  if (n < 0 || !(dt > 0.0) || !isfinite(dt)) return ORC_E_INVALID;
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 0.0) || !isfinite(L[a])) return ORC_E_INVALID;
  const double *p[3] = {x, y, z};
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (!(p[a][i] >= 0.0 && p[a][i] < L[a])) return ORC_E_INVALID;
    if (!isfinite(vx[i]) || !isfinite(vy[i]) || !isfinite(vz[i])) return ORC_E_INVALID;
    if (!(r[i] > 0.0) || !isfinite(r[i])) return ORC_E_INVALID;
    if (m && (!(m[i] > 0.0) || !isfinite(m[i]))) return ORC_E_INVALID;
  }
  return ORC_OK;
}

/*
 * Earliest partner of every active sphere over the active set (the rule stated
 * in the file header).  partner[i] = index or -1, tmin[i] = its contact time
 * (or +inf).  Inactive spheres get partner -1.
 *   use_grid = 0: all pairs, O(N^2) (the brute-force definition).
 *   use_grid = 1: candidates from the 27 surrounding cells of a grid with cell
 *                 side >= reach * cell_mult (cell_mult >= 1).
 * pair_tests (nullable) receives the number of unordered active candidate pairs.
 */
int orc_earliest(int64_t n, const double *x, const double *y, const double *z, const double *vx,
                 const double *vy, const double *vz, const double *r, const double L[3], double dt,
                 const uint8_t *active, int use_grid, double cell_mult, int64_t *partner,
                 double *tmin, int64_t *pair_tests) {
  int rc = orc_check_inputs(n, x, y, z, vx, vy, vz, r, NULL, L, dt);
  if (rc) return rc;
  const double reach = orc_reach(n, vx, vy, vz, r, dt);
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 2.0 * reach)) return ORC_E_BOX;
  if (cell_mult < 1.0) cell_mult = 1.0;
  int64_t tests2 = 0; /* ordered candidate count */
  if (!use_grid) {
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tests2)
    for (int64_t i = 0; i < n; ++i) {
      partner[i] = -1;
      tmin[i] = INFINITY;
      if (active && !active[i]) continue;
      const double xi[3] = {x[i], y[i], z[i]}, vi[3] = {vx[i], vy[i], vz[i]};
      for (int64_t j = 0; j < n; ++j) {
        if (j == i || (active && !active[j])) continue;
        ++tests2;
        const double xj[3] = {x[j], y[j], z[j]}, vj[3] = {vx[j], vy[j], vz[j]};
        double t;
        if (orc_pair_time(xi, vi, r[i], xj, vj, r[j], L, dt, &t) &&
            orc_before(t, j, tmin[i], partner[i] < 0 ? INT64_MAX : partner[i])) {
          tmin[i] = t;
          partner[i] = j;
        }
      }
    }
  } else {
    orc_grid G;
    rc = orc_grid_build(&G, n, x, y, z, vx, vy, vz, r, L, reach * cell_mult);
    if (rc) return rc;
    /* the active flags at the bucketed slots (1 = active) */
    uint8_t *sact = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!sact) {
      orc_grid_free(&G);
      return ORC_E_NOMEM;
    }
    for (int64_t k = 0; k < n; ++k) sact[k] = !active || active[G.item[k]];
    const int64_t ncell = (int64_t)G.nc[0] * G.nc[1] * G.nc[2];
    /* the particles cell by cell: each one's candidates are the particles of its
     * cell and the adjacent ones */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : tests2)
    for (int64_t c = 0; c < ncell; ++c) {
      const int c0 = (int)(c % G.nc[0]), c1 = (int)((c / G.nc[0]) % G.nc[1]),
                c2 = (int)(c / ((int64_t)G.nc[0] * G.nc[1]));
      for (int64_t s = G.start[c]; s < G.start[c + 1]; ++s) {
        const int64_t i = G.item[s];
        partner[i] = -1;
        tmin[i] = INFINITY;
        if (!sact[s]) continue;
        const double *di = G.sd + 7 * s;
        const double xi[3] = {di[0], di[1], di[2]}, vi[3] = {di[3], di[4], di[5]};
        for (int a2 = 0; a2 < G.nb[2]; ++a2)
          for (int a1 = 0; a1 < G.nb[1]; ++a1)
            for (int a0 = 0; a0 < G.nb[0]; ++a0) {
              const int64_t q = orc_neighbour(&G, c0, c1, c2, a0, a1, a2);
              for (int64_t k = G.start[q]; k < G.start[q + 1]; ++k) {
                const int64_t j = G.item[k];
                if (j == i || !sact[k]) continue;
                ++tests2;
                const double *dj = G.sd + 7 * k;
                const double xj[3] = {dj[0], dj[1], dj[2]}, vj[3] = {dj[3], dj[4], dj[5]};
                double t;
                if (orc_pair_time(xi, vi, di[6], xj, vj, dj[6], L, dt, &t) &&
                    orc_before(t, j, tmin[i], partner[i] < 0 ? INT64_MAX : partner[i])) {
                  tmin[i] = t;
                  partner[i] = j;
                }
              }
            }
      }
    }
    free(sact);
    orc_grid_free(&G);
  }
  if (pair_tests) *pair_tests = tests2 / 2;
  return ORC_OK;
}

/*
 * The same earliest-partner rule as orc_earliest, evaluated only for the
 * spheres listed in idx[0..nsub) (over all active candidates, grid search).
 * Used to check large inputs at sampled spheres.  Entries that are inactive
 * or outside [0, n) get partner -1 and time +inf.
 */
int orc_earliest_subset(int64_t n, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *r,
                        const double L[3], double dt, const uint8_t *active, int64_t nsub,
                        const int64_t *idx, int64_t *partner, double *tmin) {
  int rc = orc_check_inputs(n, x, y, z, vx, vy, vz, r, NULL, L, dt);
  if (rc) return rc;
  const double reach = orc_reach(n, vx, vy, vz, r, dt);
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 2.0 * reach)) return ORC_E_BOX;
  orc_grid G;
  rc = orc_grid_build(&G, n, x, y, z, vx, vy, vz, r, L, reach);
  if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nsub; ++s) {
    const int64_t i = idx[s];
    partner[s] = -1;
    tmin[s] = INFINITY;
    if (i < 0 || i >= n || (active && !active[i])) continue;
    const double xi[3] = {x[i], y[i], z[i]}, vi[3] = {vx[i], vy[i], vz[i]};
    const int c0 = orc_cell_of(x[i], G.h[0], G.nc[0]);
    const int c1 = orc_cell_of(y[i], G.h[1], G.nc[1]);
    const int c2 = orc_cell_of(z[i], G.h[2], G.nc[2]);
    for (int a2 = 0; a2 < G.nb[2]; ++a2)
      for (int a1 = 0; a1 < G.nb[1]; ++a1)
        for (int a0 = 0; a0 < G.nb[0]; ++a0) {
          const int64_t q = orc_neighbour(&G, c0, c1, c2, a0, a1, a2);
          for (int64_t k = G.start[q]; k < G.start[q + 1]; ++k) {
            const int64_t j = G.item[k];
            if (j == i || (active && !active[j])) continue;
            const double *dj = G.sd + 7 * k;
            const double xj[3] = {dj[0], dj[1], dj[2]}, vj[3] = {dj[3], dj[4], dj[5]};
            double t;
            if (orc_pair_time(xi, vi, r[i], xj, vj, dj[6], L, dt, &t) &&
                orc_before(t, j, tmin[s], partner[s] < 0 ? INT64_MAX : partner[s])) {
              tmin[s] = t;
              partner[s] = j;
            }
          }
        }
  }
  orc_grid_free(&G);
  return ORC_OK;
}

/* wrap one coordinate of a final position back into [0, L) (C5: one shift by L
 * suffices because no sphere moves more than L/2 in a step; a result that
 * rounds to L itself is mapped to 0) */
static double orc_wrap_pos(double p, double len) {
  if (p >= len) {
    p = p - len;
  } else if (p < 0.0) {
    p = p + len;
  }
  if (p >= len) p = 0.0;
  return p;
}

/*
 * Resolve the binary collision of spheres i and j at time t of the step,
 * Sec. "Inter-Particle Collisions" with friction 0 and eq. (update_vel1),
 * (update_vel2), (update_rho):
 *   contact separation  w = d + t u         (d, u as in orc_pair_time)
 *   unit normal i->j    n = w / s           (|w| = s at contact)
 *   normal closing rate g = u . n  (< 0)
 *   reduced mass        m_r = m_i m_j / (m_i + m_j)
 *   impulse on i        J n with J = m_r (1 + e) g, which is the paper's
 *                       J_n = -m_r (1+e) (v_r . n_p), v_r = v_i - v_j = -u
 *   velocities          v_i' = v_i + (J/m_i) n,  v_j' = v_j - (J/m_j) n
 *   positions           x' = (x + t v) + (dt - t) v'   (moved to the contact
 *                       point, then the rest of the step with v'), wrapped.
 * Reads the start-of-step state (x*, v*), writes the new state to (xo*, vo*).
 */
void orc_resolve_pair(int64_t i, int64_t j, double t, const double *x, const double *y,
                      const double *z, const double *vx, const double *vy, const double *vz,
                      const double *r, const double *m, const double L[3], double dt, double e,
                      double *xo, double *yo, double *zo, double *vxo, double *vyo, double *vzo) {
  const double xi[3] = {x[i], y[i], z[i]}, xj[3] = {x[j], y[j], z[j]};
  const double vi[3] = {vx[i], vy[i], vz[i]}, vj[3] = {vx[j], vy[j], vz[j]};
  double d[3], u[3], n[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = orc_wrap_sep(xj[k] - xi[k], L[k]);
    u[k] = vj[k] - vi[k];
  }
  const double s = r[i] + r[j];
  for (int k = 0; k < 3; ++k) {
    const double w = d[k] + t * u[k];
    n[k] = w / s;
  }
  const double g = (u[0] * n[0] + u[1] * n[1]) + u[2] * n[2];
  const double mr = (m[i] * m[j]) / (m[i] + m[j]);
  const double J = (mr * (1.0 + e)) * g;
  const double ai = J / m[i], aj = J / m[j];
  double vin[3], vjn[3];
  for (int k = 0; k < 3; ++k) {
    vin[k] = vi[k] + ai * n[k];
    vjn[k] = vj[k] - aj * n[k];
  }
  const double rest = dt - t;
  double *xout[3] = {xo, yo, zo}, *vout[3] = {vxo, vyo, vzo};
  for (int k = 0; k < 3; ++k) {
    xout[k][i] = orc_wrap_pos((xi[k] + t * vi[k]) + rest * vin[k], L[k]);
    xout[k][j] = orc_wrap_pos((xj[k] + t * vj[k]) + rest * vjn[k], L[k]);
    vout[k][i] = vin[k];
    vout[k][j] = vjn[k];
  }
}

/*
 * One side of a binary collision with friction and spin: sphere a colliding
 * with sphere b at time t, Sec. "Inter-Particle Collisions" (jump relations of
 * momentum and angular momentum, impulse J = J_n n_p + J_t t_p), taking a as
 * particle 1 (n_p points from a to b):
 *   n    = (d + t u) / s                 contact normal, d, u as in orc_pair_time
 *   J_n  = -m_r (1 + e) (v_r . n),  v_r = v_a - v_b = -u   (evaluated as
 *          (m_r (1 + e)) (u . n), the same number)
 *   v_c  = v_r + r_a w_a x n + r_b w_b x n, evaluated as v_r + (r_a w_a + r_b w_b) x n
 *          (the cross product is linear; the grouping makes the evaluation
 *          the exact negation of b's, so both sides agree to the last bit)
 *   v_rt = v_c - (v_c . n) n,  t_p = v_rt / |v_rt|
 *   J_t  = max(mu J_n, -(2/7) (1 + e) m_r |v_rt|)   (sliding, or sticking);
 *          no tangential impulse when |v_rt| = 0
 *   v_a' = v_a + J / m_a,  evaluated as v_a + (J_n/m_a) n + (J_t/m_a) t_p
 *   w_a' = w_a + (d_a/2) (n x J) / I_a = w_a + ((r_a J_t) / I_a) (n x t_p)
 *          (n x n = 0), I_a = m_a d_a^2 / 10 (a solid sphere: pi rho d^5 / 60)
 *   x_a' = (x_a + t v_a) + (dt - t) v_a'   (eq. update_rho as in orc_resolve_pair)
 * When J_t = 0 (mu = 0, or no sliding at contact) the tangential terms are
 * left out, so the result equals orc_resolve_pair's bitwise and the spin is
 * unchanged.  Reads start-of-step data; writes a's new state.
 */
static double orc_sep_axis(double d, double len, int wall);
static double orc_fly_axis(double p, double len, int wall, double *v);

/* wall: NULL for a periodic box, else the wall flags of orc_step_walls (the
 * separation of orc_sep_axis and the rest of the step flown with orc_fly_axis) */
static void orc_resolve_side_spin(int64_t a, int64_t b, double t, const double *x,
                                  const double *y, const double *z, const double *vx,
                                  const double *vy, const double *vz, const double *wx,
                                  const double *wy, const double *wz, const double *r,
                                  const double *m, const double L[3], const int *wall, double dt,
                                  double e, double mu, double *xo, double *yo, double *zo,
                                  double *vxo, double *vyo, double *vzo, double *wxo, double *wyo,
                                  double *wzo) {
  const double xa[3] = {x[a], y[a], z[a]}, xb[3] = {x[b], y[b], z[b]};
  const double va[3] = {vx[a], vy[a], vz[a]}, vb[3] = {vx[b], vy[b], vz[b]};
  const double wa[3] = {wx[a], wy[a], wz[a]}, wb[3] = {wx[b], wy[b], wz[b]};
  double d[3], u[3], n[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = wall ? orc_sep_axis(xb[k] - xa[k], L[k], wall[k]) : orc_wrap_sep(xb[k] - xa[k], L[k]);
    u[k] = vb[k] - va[k];
  }
  const double s = r[a] + r[b];
  for (int k = 0; k < 3; ++k) n[k] = (d[k] + t * u[k]) / s;
  const double g = (u[0] * n[0] + u[1] * n[1]) + u[2] * n[2];
  const double mr = (m[a] * m[b]) / (m[a] + m[b]);
  const double Jn = (mr * (1.0 + e)) * g;
  /* contact-point relative velocity and its tangential part */
  double S[3], vc[3];
  for (int k = 0; k < 3; ++k) S[k] = r[a] * wa[k] + r[b] * wb[k];
  const double Sxn[3] = {S[1] * n[2] - S[2] * n[1], S[2] * n[0] - S[0] * n[2],
                         S[0] * n[1] - S[1] * n[0]};
  for (int k = 0; k < 3; ++k) vc[k] = -u[k] + Sxn[k];
  const double vcn = (vc[0] * n[0] + vc[1] * n[1]) + vc[2] * n[2];
  double vrt[3];
  for (int k = 0; k < 3; ++k) vrt[k] = vc[k] - vcn * n[k];
  const double vt = sqrt((vrt[0] * vrt[0] + vrt[1] * vrt[1]) + vrt[2] * vrt[2]);
  double Jt = 0.0, tp[3] = {0.0, 0.0, 0.0};
  if (vt > 0.0) {
    for (int k = 0; k < 3; ++k) tp[k] = vrt[k] / vt;
    const double slide = mu * Jn;
    const double stick = -((((2.0 / 7.0) * (1.0 + e)) * mr) * vt);
    Jt = slide > stick ? slide : stick;
  }
  const double an = Jn / m[a], at = Jt / m[a];
  double van[3];
  for (int k = 0; k < 3; ++k) {
    van[k] = va[k] + an * n[k];
    if (Jt != 0.0) van[k] = van[k] + at * tp[k];
  }
  const double rest = dt - t;
  double *xout[3] = {xo, yo, zo}, *vout[3] = {vxo, vyo, vzo}, *wout[3] = {wxo, wyo, wzo};
  for (int k = 0; k < 3; ++k) {
    double vk = van[k];
    xout[k][a] = wall ? orc_fly_axis((xa[k] + t * va[k]) + rest * van[k], L[k], wall[k], &vk)
                      : orc_wrap_pos((xa[k] + t * va[k]) + rest * van[k], L[k]);
    vout[k][a] = vk;
    wout[k][a] = wa[k];
  }
  if (Jt != 0.0) {
    const double da = 2.0 * r[a];
    const double I = (m[a] * (da * da)) / 10.0;
    const double K = (r[a] * Jt) / I;
    const double nxt[3] = {n[1] * tp[2] - n[2] * tp[1], n[2] * tp[0] - n[0] * tp[2],
                           n[0] * tp[1] - n[1] * tp[0]};
    for (int k = 0; k < 3; ++k) wout[k][a] = wa[k] + K * nxt[k];
  }
}

/* Both sides of the collision of i and j at time t, with friction and spin. */
void orc_resolve_pair_spin(int64_t i, int64_t j, double t, const double *x, const double *y,
                           const double *z, const double *vx, const double *vy,
                           const double *vz, const double *wx, const double *wy,
                           const double *wz, const double *r, const double *m,
                           const double L[3], double dt, double e, double mu, double *xo,
                           double *yo, double *zo, double *vxo, double *vyo, double *vzo,
                           double *wxo, double *wyo, double *wzo) {
  orc_resolve_side_spin(i, j, t, x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, NULL, dt, e, mu, xo, yo, zo,
                        vxo, vyo, vzo, wxo, wyo, wzo);
  orc_resolve_side_spin(j, i, t, x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, NULL, dt, e, mu, xo, yo, zo,
                        vxo, vyo, vzo, wxo, wyo, wzo);
}

typedef struct {
  int64_t n_pairs;    /* collisions resolved in the step */
  int64_t n_sweeps;   /* sweeps run, including the final one that found none */
  int64_t pair_tests; /* unordered active candidate pairs, summed over sweeps */
  double reach;
} orc_stats;

/*
 * One full collision step (the sweeps described in the file header), Sec.
 * "Collision Operator": detect over the eligible set, resolve mutual earliest
 * pairs, remove them from the eligible set, repeat; then free flight and wrap.
 * Inputs (x*, v*, r, m) are the start-of-step state and are not modified; the
 * new state goes to (xo*, vo*).  partner[i] = the sphere i collided with or -1;
 * tcoll[i] = contact time within the step (NaN if none); sweep_of[i] = sweep
 * (0-based) in which i collided, or -1.  Any of the three may be NULL.  With
 * spins (w* not NULL) the resolve also applies friction mu and writes the new
 * spins to (wo*); without, it is the frictionless orc_resolve_pair.
 */
static int orc_step_core(int64_t n, const double *x, const double *y, const double *z,
                         const double *vx, const double *vy, const double *vz, const double *wx,
                         const double *wy, const double *wz, const double *r, const double *m,
                         const double L[3], double dt, double e, double mu, int use_grid,
                         double cell_mult, int max_sweeps, double *xo, double *yo, double *zo,
                         double *vxo, double *vyo, double *vzo, double *wxo, double *wyo,
                         double *wzo, int64_t *partner, double *tcoll, int32_t *sweep_of,
                         orc_stats *st) {
  int rc = orc_check_inputs(n, x, y, z, vx, vy, vz, r, m, L, dt);
  if (rc) return rc;
  if (!(e >= 0.0 && e <= 1.0)) return ORC_E_INVALID;
  if (wx) {
    if (!(mu >= 0.0) || !isfinite(mu)) return ORC_E_INVALID;
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(wx[i]) || !isfinite(wy[i]) || !isfinite(wz[i])) return ORC_E_INVALID;
  }
  const double reach = orc_reach(n, vx, vy, vz, r, dt);
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 2.0 * reach)) return ORC_E_BOX;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  uint8_t *active = (uint8_t *)malloc(nn);
  uint8_t *hit = (uint8_t *)malloc(nn);
  int64_t *pj = (int64_t *)malloc(nn * sizeof(int64_t));
  double *pt = (double *)malloc(nn * sizeof(double));
  if (!active || !hit || !pj || !pt) {
    free(active);
    free(hit);
    free(pj);
    free(pt);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    active[i] = 1;
    hit[i] = 0;
    if (partner) partner[i] = -1;
    if (tcoll) tcoll[i] = NAN;
    if (sweep_of) sweep_of[i] = -1;
  }
  int64_t pairs = 0, tests = 0, sweeps = 0;
  for (;;) {
    int64_t tk = 0;
    rc = orc_earliest(n, x, y, z, vx, vy, vz, r, L, dt, active, use_grid, cell_mult, pj, pt, &tk);
    if (rc) break;
    tests += tk;
    ++sweeps;
    int64_t found = 0;
#pragma omp parallel for schedule(static) reduction(+ : found)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = pj[i];
      if (j > i && pj[j] == i) {
        if (wx)
          orc_resolve_pair_spin(i, j, pt[i], x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, dt, e, mu,
                                xo, yo, zo, vxo, vyo, vzo, wxo, wyo, wzo);
        else
          orc_resolve_pair(i, j, pt[i], x, y, z, vx, vy, vz, r, m, L, dt, e, xo, yo, zo, vxo,
                           vyo, vzo);
        hit[i] = hit[j] = 1;
        if (partner) {
          partner[i] = j;
          partner[j] = i;
        }
        if (tcoll) tcoll[i] = tcoll[j] = pt[i];
        if (sweep_of) sweep_of[i] = sweep_of[j] = (int32_t)(sweeps - 1);
        ++found;
      }
    }
    if (found == 0) break;
    pairs += found;
    for (int64_t i = 0; i < n; ++i)
      if (hit[i]) active[i] = 0;
    if (max_sweeps > 0 && sweeps >= max_sweeps) {
      rc = ORC_E_SWEEPS;
      break;
    }
  }
  if (rc == ORC_OK) {
    const double *p[3] = {x, y, z}, *v[3] = {vx, vy, vz};
    double *po[3] = {xo, yo, zo}, *vo[3] = {vxo, vyo, vzo};
    for (int64_t i = 0; i < n; ++i) {
      if (hit[i]) continue;
      for (int k = 0; k < 3; ++k) {
        po[k][i] = orc_wrap_pos(p[k][i] + dt * v[k][i], L[k]);
        vo[k][i] = v[k][i];
      }
      if (wx) {
        wxo[i] = wx[i];
        wyo[i] = wy[i];
        wzo[i] = wz[i];
      }
    }
  }
  if (st) {
    st->n_pairs = pairs;
    st->n_sweeps = sweeps;
    st->pair_tests = tests;
    st->reach = reach;
  }
  free(active);
  free(hit);
  free(pj);
  free(pt);
  return rc;
}

/* One collision step without friction (see orc_step_core). */
int orc_step(int64_t n, const double *x, const double *y, const double *z, const double *vx,
             const double *vy, const double *vz, const double *r, const double *m,
             const double L[3], double dt, double e, int use_grid, double cell_mult, int max_sweeps,
             double *xo, double *yo, double *zo, double *vxo, double *vyo, double *vzo,
             int64_t *partner, double *tcoll, int32_t *sweep_of, orc_stats *st) {
  return orc_step_core(n, x, y, z, vx, vy, vz, NULL, NULL, NULL, r, m, L, dt, e, 0.0, use_grid,
                       cell_mult, max_sweeps, xo, yo, zo, vxo, vyo, vzo, NULL, NULL, NULL,
                       partner, tcoll, sweep_of, st);
}

/* One collision step with angular velocities (w*) and Coulomb friction mu
 * (orc_resolve_side_spin); the new spins go to (wo*).  The pair set is the one
 * of orc_step: contact times do not depend on the spins. */
int orc_step_spin(int64_t n, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz, const double *wx,
                  const double *wy, const double *wz, const double *r, const double *m,
                  const double L[3], double dt, double e, double mu, int use_grid,
                  double cell_mult, int max_sweeps, double *xo, double *yo, double *zo,
                  double *vxo, double *vyo, double *vzo, double *wxo, double *wyo, double *wzo,
                  int64_t *partner, double *tcoll, int32_t *sweep_of, orc_stats *st) {
  if (n > 0 && (!wx || !wy || !wz || !wxo || !wyo || !wzo)) return ORC_E_INVALID;
  return orc_step_core(n, x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, dt, e, mu, use_grid,
                       cell_mult, max_sweeps, xo, yo, zo, vxo, vyo, vzo, wxo, wyo, wzo, partner,
                       tcoll, sweep_of, st);
}

/*
 * Forward-mode derivative (Jacobian-vector product) of one step with the pair
 * set held fixed at the primal's: the same sweeps pick the pairs, then every
 * quantity of the resolve carries a tangent (Sec. "Inter-Particle Collisions"
 * and eq. update_vel/update_rho differentiated by hand).
 *
 * For a pair (i, j) with d = x_j - x_i, u = v_j - v_i, contact time t, w = d + t u,
 * n = w / s, g = u . n, c = m_r (1 + e), J = c g:
 *   the contact condition |w|^2 = s^2 gives  t' = -(n . d' + t n . u') / g,
 *   w' = d' + t u' + t' u,  n' = w' / s,  g' = u' . n + u . n',
 *   J' = c g' + m_r g e',
 *   v_i' -> v_i' + (J'/m_i) n + (J/m_i) n',   v_j' -> v_j' - (J'/m_j) n - (J/m_j) n',
 *   x_i' -> x_i' + t' (v_i - v_i_new) + t v_i' + (dt - t) v_i_new'.
 * Spheres without a collision: x' = x + dt v'  (tangent), v' unchanged.
 * Periodic wraps shift by constants and do not enter the tangents.
 * Tangent inputs dx, dy, dz, dvx, dvy, dvz (arrays) and de; tangent outputs
 * tx.., tv... Also writes the primal like orc_step.
 */
int orc_step_jvp(int64_t n, const double *x, const double *y, const double *z, const double *vx,
                 const double *vy, const double *vz, const double *r, const double *m,
                 const double L[3], double dt, double e, const double *dx, const double *dy,
                 const double *dz, const double *dvx, const double *dvy, const double *dvz,
                 double de, double *xo, double *yo, double *zo, double *vxo, double *vyo,
                 double *vzo, double *txo, double *tyo, double *tzo, double *tvxo, double *tvyo,
                 double *tvzo, int64_t *partner) {
  const size_t nn = (size_t)(n > 0 ? n : 1);
  double *tc = (double *)malloc(nn * sizeof(double));
  int64_t *pp = partner ? partner : (int64_t *)malloc(nn * sizeof(int64_t));
  if (!tc || !pp) {
    free(tc);
    if (!partner) free(pp);
    return ORC_E_NOMEM;
  }
  int rc = orc_step(n, x, y, z, vx, vy, vz, r, m, L, dt, e, 1, 1.0, 0, xo, yo, zo, vxo, vyo, vzo,
                    pp, tc, NULL, NULL);
  if (rc == ORC_OK) {
    const double *X[3] = {x, y, z}, *V[3] = {vx, vy, vz};
    const double *DX[3] = {dx, dy, dz}, *DV[3] = {dvx, dvy, dvz};
    double *TX[3] = {txo, tyo, tzo}, *TV[3] = {tvxo, tvyo, tvzo};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = pp[i];
      if (j < 0) {
        for (int k = 0; k < 3; ++k) {
          TX[k][i] = DX[k][i] + dt * DV[k][i];
          TV[k][i] = DV[k][i];
        }
        continue;
      }
      /* primal of the pair from i's side (n points from i to j) */
      const double t = tc[i];
      double d[3], u[3], w[3], nv[3];
      for (int k = 0; k < 3; ++k) {
        d[k] = orc_wrap_sep(X[k][j] - X[k][i], L[k]);
        u[k] = V[k][j] - V[k][i];
      }
      const double s = r[i] + r[j];
      for (int k = 0; k < 3; ++k) {
        w[k] = d[k] + t * u[k];
        nv[k] = w[k] / s;
      }
      const double g = (u[0] * nv[0] + u[1] * nv[1]) + u[2] * nv[2];
      const double mr = (m[i] * m[j]) / (m[i] + m[j]);
      const double c = mr * (1.0 + e);
      const double J = c * g;
      /* tangents */
      double dd[3], du[3];
      for (int k = 0; k < 3; ++k) {
        dd[k] = DX[k][j] - DX[k][i];
        du[k] = DV[k][j] - DV[k][i];
      }
      const double nd = nv[0] * dd[0] + nv[1] * dd[1] + nv[2] * dd[2];
      const double nu = nv[0] * du[0] + nv[1] * du[1] + nv[2] * du[2];
      const double tt = -(nd + t * nu) / g;
      double dn[3];
      for (int k = 0; k < 3; ++k) dn[k] = (dd[k] + t * du[k] + tt * u[k]) / s;
      const double dg = (du[0] * nv[0] + du[1] * nv[1] + du[2] * nv[2]) +
                        (u[0] * dn[0] + u[1] * dn[1] + u[2] * dn[2]);
      const double dJ = c * dg + mr * g * de;
      for (int k = 0; k < 3; ++k) {
        const double vnew = V[k][i] + (J / m[i]) * nv[k];
        const double dvnew = DV[k][i] + (dJ / m[i]) * nv[k] + (J / m[i]) * dn[k];
        TV[k][i] = dvnew;
        TX[k][i] = DX[k][i] + tt * (V[k][i] - vnew) + t * DV[k][i] + (dt - t) * dvnew;
      }
    }
  }
  free(tc);
  if (!partner) free(pp);
  return rc;
}

/*
 * Deposition of a per-sphere quantity onto the corner nodes of a periodic
 * Cartesian grid, Sec. "Dispersed Phase" (projection operator onto the corner
 * nodes of the host element) and Sec. "Deposition" (linear deposition with
 * radius equal to the cell size, conservative).  The grid has nc[d] cells of
 * side h[d] = L[d] / nc[d] per axis and one node per cell corner, node (i, j, k)
 * at (i h0, j h1, k h2), numbered (k nc1 + j) nc0 + i, indices periodic.  A
 * sphere at x in cell c (c[d] = floor(x[d] / h[d]), clamped to nc[d] - 1) with
 * local coordinate f[d] = x[d] / h[d] - c[d] in [0, 1] gives node
 * c + (b0, b1, b2), b in {0, 1}^3, the weight
 *   w = prod_d (b_d ? f_d : 1 - f_d),
 * which on cells of equal volume is the linear (C0) corner weighting of the
 * paper's operator: the weights of a sphere sum to 1 and reproduce linear
 * fields.  comp components per sphere, a[q * n + i]; out[q * nnode + node]
 * receives the sums (overwritten).  Spheres are added in index order, the
 * eight corners in the order b0 fastest.
 */
int orc_deposit(int64_t n, const double *x, const double *y, const double *z, const double *a,
                int comp, const int nc[3], const double L[3], double *out) {
  if (n < 0 || comp < 1) return ORC_E_INVALID;
  for (int d = 0; d < 3; ++d)
    if (nc[d] < 1 || !(L[d] > 0.0)) return ORC_E_INVALID;
  const int64_t nnode = (int64_t)nc[0] * nc[1] * nc[2];
  for (int64_t k = 0; k < nnode * comp; ++k) out[k] = 0.0;
  const double h[3] = {L[0] / nc[0], L[1] / nc[1], L[2] / nc[2]};
  for (int64_t i = 0; i < n; ++i) {
    const double p[3] = {x[i], y[i], z[i]};
    int c[3];
    double f[3];
    for (int d = 0; d < 3; ++d) {
      if (!isfinite(p[d]) || !(p[d] >= 0.0 && p[d] < L[d])) return ORC_E_INVALID;
      const double s = p[d] / h[d];
      int cd = (int)floor(s);
      if (cd > nc[d] - 1) cd = nc[d] - 1;
      c[d] = cd;
      f[d] = s - (double)cd;
    }
    for (int b = 0; b < 8; ++b) {
      const int b0 = b & 1, b1 = (b >> 1) & 1, b2 = (b >> 2) & 1;
      const double w = ((b0 ? f[0] : 1.0 - f[0]) * (b1 ? f[1] : 1.0 - f[1])) *
                       (b2 ? f[2] : 1.0 - f[2]);
      const int ix = (c[0] + b0) % nc[0], iy = (c[1] + b1) % nc[1], iz = (c[2] + b2) % nc[2];
      const int64_t node = ((int64_t)iz * nc[1] + iy) * nc[0] + ix;
      for (int q = 0; q < comp; ++q) out[(int64_t)q * nnode + node] += w * a[(int64_t)q * n + i];
    }
  }
  return ORC_OK;
}

/* Morton (Z-order) key of a cell: bits of cx, cy, cz interleaved, x lowest. */
static uint64_t orc_morton(int cx, int cy, int cz) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b) {
    k |= (uint64_t)((cx >> b) & 1) << (3 * b);
    k |= (uint64_t)((cy >> b) & 1) << (3 * b + 1);
    k |= (uint64_t)((cz >> b) & 1) << (3 * b + 2);
  }
  return k;
}

typedef struct {
  uint64_t key;
  int64_t cell;
} orc_keyed;

static int orc_keyed_cmp(const void *a, const void *b) {
  const orc_keyed *p = (const orc_keyed *)a, *q = (const orc_keyed *)b;
  return p->key < q->key ? -1 : (p->key > q->key ? 1 : 0);
}

/*
 * One step with the collision order of the paper taken literally, Sec.
 * "Collision Operator" and Sec. "Particle-Particle Collisions": the elements
 * (here the cells of the plain grid, side >= reach * cell_mult) are visited in
 * the order of a space-filling curve (Morton order: the paper names none); the
 * particles of an element in index order; each still eligible particle i scans
 * its candidate elements (its own and the adjacent ones, periodic, sorted along
 * the same curve), their particles in index order, and the first eligible j
 * whose contact time (orc_pair_time: two positive roots, approach, t <= dt)
 * exists is its partner: both are resolved at once (orc_resolve_pair, from
 * start-of-step data) and leave the eligible set.  Every particle without a
 * collision flies freely.  One pass, no sweeps; the result is a maximal set
 * of disjoint colliding pairs, not in general the earliest-partner set.
 * Outputs as orc_step; st->n_sweeps = 1, st->pair_tests counts contact-time
 * evaluations.
 */
int orc_step_sequential(int64_t n, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *r,
                        const double *m, const double L[3], double dt, double e, double cell_mult,
                        double *xo, double *yo, double *zo, double *vxo, double *vyo,
                        double *vzo, int64_t *partner, double *tcoll, orc_stats *st) {
  int rc = orc_check_inputs(n, x, y, z, vx, vy, vz, r, m, L, dt);
  if (rc) return rc;
  if (!(e >= 0.0 && e <= 1.0) || !(cell_mult >= 1.0)) return ORC_E_INVALID;
  const double reach = orc_reach(n, vx, vy, vz, r, dt);
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 2.0 * reach)) return ORC_E_BOX;
  orc_grid G;
  rc = orc_grid_build(&G, n, x, y, z, vx, vy, vz, r, L, reach * cell_mult);
  if (rc) return rc;
  const int64_t ncell = (int64_t)G.nc[0] * G.nc[1] * G.nc[2];
  orc_keyed *order = (orc_keyed *)malloc((size_t)(ncell > 0 ? ncell : 1) * sizeof(orc_keyed));
  uint8_t *hit = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!order || !hit) {
    free(order);
    free(hit);
    orc_grid_free(&G);
    return ORC_E_NOMEM;
  }
  for (int64_t c = 0; c < ncell; ++c) {
    const int cx = (int)(c % G.nc[0]), cy = (int)((c / G.nc[0]) % G.nc[1]),
              cz = (int)(c / ((int64_t)G.nc[0] * G.nc[1]));
    order[c].key = orc_morton(cx, cy, cz);
    order[c].cell = c;
  }
  qsort(order, (size_t)ncell, sizeof(orc_keyed), orc_keyed_cmp);
  for (int64_t i = 0; i < n; ++i) {
    if (partner) partner[i] = -1;
    if (tcoll) tcoll[i] = NAN;
  }
  int64_t pairs = 0, tests = 0;
  for (int64_t oc = 0; oc < ncell; ++oc) {
    const int64_t c = order[oc].cell;
    const int cx = (int)(c % G.nc[0]), cy = (int)((c / G.nc[0]) % G.nc[1]),
              cz = (int)(c / ((int64_t)G.nc[0] * G.nc[1]));
    /* candidate elements of this element, sorted along the curve */
    orc_keyed cand[27];
    int nk = 0;
    for (int a = 0; a < G.nb[2]; ++a)
      for (int b = 0; b < G.nb[1]; ++b)
        for (int d = 0; d < G.nb[0]; ++d) {
          const int qx = (cx + G.off[0][d] + G.nc[0]) % G.nc[0];
          const int qy = (cy + G.off[1][b] + G.nc[1]) % G.nc[1];
          const int qz = (cz + G.off[2][a] + G.nc[2]) % G.nc[2];
          cand[nk].key = orc_morton(qx, qy, qz);
          cand[nk].cell = ((int64_t)qz * G.nc[1] + qy) * G.nc[0] + qx;
          ++nk;
        }
    qsort(cand, (size_t)nk, sizeof(orc_keyed), orc_keyed_cmp);
    for (int64_t s = G.start[c]; s < G.start[c + 1]; ++s) {
      const int64_t i = G.item[s];
      if (hit[i]) continue;
      const double xi[3] = {x[i], y[i], z[i]}, vi[3] = {vx[i], vy[i], vz[i]};
      for (int k = 0; k < nk && !hit[i]; ++k) {
        const int64_t q = cand[k].cell;
        for (int64_t u = G.start[q]; u < G.start[q + 1]; ++u) {
          const int64_t j = G.item[u];
          if (j == i || hit[j]) continue;
          const double *dj = G.sd + 7 * u;
          const double xj[3] = {dj[0], dj[1], dj[2]}, vj[3] = {dj[3], dj[4], dj[5]};
          double t;
          ++tests;
          if (!orc_pair_time(xi, vi, r[i], xj, vj, dj[6], L, dt, &t)) continue;
          orc_resolve_pair(i, j, t, x, y, z, vx, vy, vz, r, m, L, dt, e, xo, yo, zo, vxo, vyo,
                           vzo);
          hit[i] = hit[j] = 1;
          if (partner) {
            partner[i] = j;
            partner[j] = i;
          }
          if (tcoll) tcoll[i] = tcoll[j] = t;
          ++pairs;
          break;
        }
      }
    }
  }
  const double *p[3] = {x, y, z}, *v[3] = {vx, vy, vz};
  double *po[3] = {xo, yo, zo}, *vo[3] = {vxo, vyo, vzo};
  for (int64_t i = 0; i < n; ++i) {
    if (hit[i]) continue;
    for (int k = 0; k < 3; ++k) {
      po[k][i] = orc_wrap_pos(p[k][i] + dt * v[k][i], L[k]);
      vo[k][i] = v[k][i];
    }
  }
  if (st) {
    st->n_pairs = pairs;
    st->n_sweeps = 1;
    st->pair_tests = tests;
    st->reach = reach;
  }
  free(order);
  free(hit);
  orc_grid_free(&G);
  return ORC_OK;
}

/* ---------------------------------------------------------------- walls */

/* separation along one axis: the minimum image on a periodic axis, the plain
 * difference between two walls */
static double orc_sep_axis(double d, double len, int wall) {
  return wall ? d : orc_wrap_sep(d, len);
}

/* Time of flight of a centre at x with velocity v until it reaches a wall plane
 * (x_k = 0 or x_k = L_k on a wall axis), +inf if it moves along no wall axis:
 * Sec. "Particle-Particle Collisions" (each particle's time of flight to its
 * next boundary intersection) with the particle tracked by its centre. */
static double orc_time_to_wall(const double x[3], const double v[3], const double L[3],
                               const int wall[3]) {
  double tw = INFINITY;
  for (int k = 0; k < 3; ++k) {
    if (!wall[k]) continue;
    double t;
    if (v[k] > 0.0)
      t = (L[k] - x[k]) / v[k];
    else if (v[k] < 0.0)
      t = -x[k] / v[k];
    else
      continue;
    if (t < tw) tw = t;
  }
  return tw;
}

/* Contact time of spheres i and j as orc_pair_time, with the separation of
 * orc_sep_axis, and valid only if it is no later than either sphere's time of
 * flight to a wall (Sec. "Particle Collisions": the collision must occur
 * before an intersection with a domain boundary). */
static int orc_pair_time_walls(const double xi[3], const double vi[3], double ri,
                               const double xj[3], const double vj[3], double rj,
                               const double L[3], const int wall[3], double dt, double *t_out) {
  double d[3], u[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = orc_sep_axis(xj[k] - xi[k], L[k], wall[k]);
    u[k] = vj[k] - vi[k];
  }
  const double s = ri + rj;
  const double a = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
  const double b = (d[0] * u[0] + d[1] * u[1]) + d[2] * u[2];
  const double c = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) - s * s;
  if (!(a > 0.0) || !(b < 0.0) || !(c > 0.0)) return 0;
  const double D = b * b - a * c;
  if (!(D >= 0.0)) return 0;
  const double t = c / (-b + sqrt(D));
  if (!(t <= dt)) return 0;
  if (!(t <= orc_time_to_wall(xi, vi, L, wall)) || !(t <= orc_time_to_wall(xj, vj, L, wall)))
    return 0;
  *t_out = t;
  return 1;
}

/* End of a flight along one axis: p is the unconstrained coordinate.  On a
 * periodic axis it is wrapped (orc_wrap_pos).  On a wall axis a centre beyond a
 * wall plane is reflected at it, Sec. "Intersection of Particles with Solid
 * Walls" with a perfectly reflective wall (momentum change zero: the normal
 * velocity component changes sign, the spin is unchanged); at most one plane is
 * crossed because no sphere moves more than L/4 in a step.  A coordinate that
 * lands on L itself becomes the largest double below L. */
static double orc_fly_axis(double p, double len, int wall, double *v) {
  if (!wall) return orc_wrap_pos(p, len);
  if (p >= len) {
    p = len - (p - len);
    *v = -*v;
  } else if (p < 0.0) {
    p = -p;
    *v = -*v;
  }
  if (p >= len) p = nextafter(len, 0.0);
  return p;
}

/* Resolve of the pair (i, j) at time t as orc_resolve_pair, with the
 * separation of orc_sep_axis and the rest of the step flown with orc_fly_axis. */
static void orc_resolve_pair_walls(int64_t i, int64_t j, double t, const double *x,
                                   const double *y, const double *z, const double *vx,
                                   const double *vy, const double *vz, const double *r,
                                   const double *m, const double L[3], const int wall[3],
                                   double dt, double e, double *xo, double *yo, double *zo,
                                   double *vxo, double *vyo, double *vzo) {
  const double xi[3] = {x[i], y[i], z[i]}, xj[3] = {x[j], y[j], z[j]};
  const double vi[3] = {vx[i], vy[i], vz[i]}, vj[3] = {vx[j], vy[j], vz[j]};
  double d[3], u[3], nrm[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = orc_sep_axis(xj[k] - xi[k], L[k], wall[k]);
    u[k] = vj[k] - vi[k];
  }
  const double s = r[i] + r[j];
  for (int k = 0; k < 3; ++k) nrm[k] = (d[k] + t * u[k]) / s;
  const double g = (u[0] * nrm[0] + u[1] * nrm[1]) + u[2] * nrm[2];
  const double mr = (m[i] * m[j]) / (m[i] + m[j]);
  const double J = (mr * (1.0 + e)) * g;
  const double ai = J / m[i], aj = J / m[j];
  const double rest = dt - t;
  double *xout[3] = {xo, yo, zo}, *vout[3] = {vxo, vyo, vzo};
  for (int k = 0; k < 3; ++k) {
    double vin = vi[k] + ai * nrm[k];
    double vjn = vj[k] - aj * nrm[k];
    xout[k][i] = orc_fly_axis((xi[k] + t * vi[k]) + rest * vin, L[k], wall[k], &vin);
    xout[k][j] = orc_fly_axis((xj[k] + t * vj[k]) + rest * vjn, L[k], wall[k], &vjn);
    vout[k][i] = vin;
    vout[k][j] = vjn;
  }
}

/*
 * One collision step with reflective walls on the axes where wall[k] != 0 (the
 * other axes periodic): the rule of orc_step with the pair time of
 * orc_pair_time_walls, the resolve of orc_resolve_pair_walls and the free flight
 * of orc_fly_axis.  Candidates come from the plain grid with periodic
 * neighbours: a pair that is neighbours only through a wall is at least a cell
 * side (>= reach) apart without the minimum image and cannot touch within the
 * step.  Outputs and errors as orc_step.
 */
static int orc_step_walls_core(int64_t n, const double *x, const double *y, const double *z,
                               const double *vx, const double *vy, const double *vz,
                               const double *wx, const double *wy, const double *wz,
                               const double *r, const double *m, const double L[3],
                               const int wall[3], double dt, double e, double mu, double *xo,
                               double *yo, double *zo, double *vxo, double *vyo, double *vzo,
                               double *wxo, double *wyo, double *wzo, int64_t *partner,
                               double *tcoll, orc_stats *st) {
  int rc = orc_check_inputs(n, x, y, z, vx, vy, vz, r, m, L, dt);
  if (rc) return rc;
  if (!(e >= 0.0 && e <= 1.0)) return ORC_E_INVALID;
  if (wx) {
    if (!(mu >= 0.0) || !isfinite(mu)) return ORC_E_INVALID;
    for (int64_t i = 0; i < n; ++i)
      if (!isfinite(wx[i]) || !isfinite(wy[i]) || !isfinite(wz[i])) return ORC_E_INVALID;
  }
  const double reach = orc_reach(n, vx, vy, vz, r, dt);
  for (int a = 0; a < 3; ++a)
    if (!(L[a] > 2.0 * reach)) return ORC_E_BOX;
  orc_grid G;
  rc = orc_grid_build(&G, n, x, y, z, vx, vy, vz, r, L, reach);
  if (rc) return rc;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  uint8_t *hit = (uint8_t *)calloc(nn, 1);
  int64_t *pj = (int64_t *)malloc(nn * sizeof(int64_t));
  double *pt = (double *)malloc(nn * sizeof(double));
  if (!hit || !pj || !pt) {
    free(hit);
    free(pj);
    free(pt);
    orc_grid_free(&G);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (partner) partner[i] = -1;
    if (tcoll) tcoll[i] = NAN;
  }
  int64_t pairs = 0, tests = 0, sweeps = 0;
  for (;;) {
    int64_t tk = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tk)
    for (int64_t i = 0; i < n; ++i) {
      pj[i] = -1;
      pt[i] = INFINITY;
      if (hit[i]) continue;
      const double xi[3] = {x[i], y[i], z[i]}, vi[3] = {vx[i], vy[i], vz[i]};
      const int c0 = orc_cell_of(x[i], G.h[0], G.nc[0]);
      const int c1 = orc_cell_of(y[i], G.h[1], G.nc[1]);
      const int c2 = orc_cell_of(z[i], G.h[2], G.nc[2]);
      for (int a2 = 0; a2 < G.nb[2]; ++a2)
        for (int a1 = 0; a1 < G.nb[1]; ++a1)
          for (int a0 = 0; a0 < G.nb[0]; ++a0) {
            const int q0 = (c0 + G.off[0][a0] + G.nc[0]) % G.nc[0];
            const int q1 = (c1 + G.off[1][a1] + G.nc[1]) % G.nc[1];
            const int q2 = (c2 + G.off[2][a2] + G.nc[2]) % G.nc[2];
            const int64_t q = ((int64_t)q2 * G.nc[1] + q1) * G.nc[0] + q0;
            for (int64_t k = G.start[q]; k < G.start[q + 1]; ++k) {
              const int64_t j = G.item[k];
              if (j == i || hit[j]) continue;
              ++tk;
              const double *dj = G.sd + 7 * k;
              const double xj[3] = {dj[0], dj[1], dj[2]}, vj[3] = {dj[3], dj[4], dj[5]};
              double t;
              if (orc_pair_time_walls(xi, vi, r[i], xj, vj, dj[6], L, wall, dt, &t) &&
                  orc_before(t, j, pt[i], pj[i] < 0 ? INT64_MAX : pj[i])) {
                pt[i] = t;
                pj[i] = j;
              }
            }
          }
    }
    tests += tk / 2;
    ++sweeps;
    int64_t found = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = pj[i];
      if (j > i && pj[j] == i) {
        if (wx) {
          orc_resolve_side_spin(i, j, pt[i], x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, wall, dt, e,
                                mu, xo, yo, zo, vxo, vyo, vzo, wxo, wyo, wzo);
          orc_resolve_side_spin(j, i, pt[i], x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, wall, dt, e,
                                mu, xo, yo, zo, vxo, vyo, vzo, wxo, wyo, wzo);
        } else {
          orc_resolve_pair_walls(i, j, pt[i], x, y, z, vx, vy, vz, r, m, L, wall, dt, e, xo, yo,
                                 zo, vxo, vyo, vzo);
        }
        if (partner) {
          partner[i] = j;
          partner[j] = i;
        }
        if (tcoll) tcoll[i] = tcoll[j] = pt[i];
        ++found;
      }
    }
    if (found == 0) break;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = pj[i];
      if (j >= 0 && pj[j] == i) hit[i] = 1;
    }
    pairs += found;
  }
  const double *p[3] = {x, y, z}, *v[3] = {vx, vy, vz};
  double *po[3] = {xo, yo, zo}, *vo[3] = {vxo, vyo, vzo};
  for (int64_t i = 0; i < n; ++i) {
    if (hit[i]) continue;
    for (int k = 0; k < 3; ++k) {
      double vk = v[k][i];
      po[k][i] = orc_fly_axis(p[k][i] + dt * vk, L[k], wall[k], &vk);
      vo[k][i] = vk;
    }
    if (wx) { /* an elastic wall leaves the spin unchanged */
      wxo[i] = wx[i];
      wyo[i] = wy[i];
      wzo[i] = wz[i];
    }
  }
  if (st) {
    st->n_pairs = pairs;
    st->n_sweeps = sweeps;
    st->pair_tests = tests;
    st->reach = reach;
  }
  free(hit);
  free(pj);
  free(pt);
  orc_grid_free(&G);
  return ORC_OK;
}

/* One step between walls without friction (orc_step_walls_core). */
int orc_step_walls(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *r,
                   const double *m, const double L[3], const int wall[3], double dt, double e,
                   double *xo, double *yo, double *zo, double *vxo, double *vyo, double *vzo,
                   int64_t *partner, double *tcoll, orc_stats *st) {
  return orc_step_walls_core(n, x, y, z, vx, vy, vz, NULL, NULL, NULL, r, m, L, wall, dt, e, 0.0,
                             xo, yo, zo, vxo, vyo, vzo, NULL, NULL, NULL, partner, tcoll, st);
}

/* One step between walls with spins and Coulomb friction mu: the pair resolve
 * of orc_step_spin (orc_resolve_side_spin) with the separation and flight of
 * the walls; an elastic wall leaves the spin unchanged (its momentum change is
 * zero, so the angular jump relation of Sec. "Intersection of Particles with
 * Solid Walls" gives no spin change). */
int orc_step_walls_spin(int64_t n, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *wx,
                        const double *wy, const double *wz, const double *r, const double *m,
                        const double L[3], const int wall[3], double dt, double e, double mu,
                        double *xo, double *yo, double *zo, double *vxo, double *vyo,
                        double *vzo, double *wxo, double *wyo, double *wzo, int64_t *partner,
                        double *tcoll, orc_stats *st) {
  return orc_step_walls_core(n, x, y, z, vx, vy, vz, wx, wy, wz, r, m, L, wall, dt, e, mu, xo, yo,
                             zo, vxo, vyo, vzo, wxo, wyo, wzo, partner, tcoll, st);
}
