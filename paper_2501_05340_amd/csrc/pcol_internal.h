// Internal declarations of the pcol HIP library: device helpers shared by the
// kernels and the launch wrappers the C-ABI layer calls.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace pcol {

// Cell-sorted start-of-step record of one sphere (64 B, one HBM burst).  It
// carries the sphere's caller index o (the tie-break key of the partner rule and
// the output position) and its box in the batched form, so binning writes one
// record per sphere and nothing else in sorted order; the mass, needed only
// for a collision, is read from the caller's array at o.
struct alignas(16) Rec {
  double x, y, z, r;
  double vx, vy, vz;
  int o;    // caller index
  int box;  // box of the batched form (0 otherwise)
};

// Sphere status during a step: ACTIVE has a valid partner key (or none yet),
// DIRTY is active but its partner collided with another sphere, so its key
// must be recomputed; FREE has no contact left in the step; COLLIDED is done.
enum : uint8_t { ST_ACTIVE = 0, ST_FREE = 1, ST_COLLIDED = 2, ST_DIRTY = 3 };

// End-of-step state of one collided sphere in cell-sorted order (64 B), copied
// to the caller's order by a final gather.
struct alignas(16) OutRec {
  double x, y, z, vx, vy, vz, t;
  int partner;          // caller index
  unsigned int pad;
};

// Uniform grid over the periodic box.  Cells are numbered (cz * nc1 + cy) * nc0 + cx,
// so the cells of one x-row are consecutive and so are their spheres after sorting.
//
// With the extent split (see k_cell_hist) the spheres of large extent sit in a
// second layer of the same cells, numbered layer2 + c; layer2 = 0 means one
// layer.  rho_max > 0 is the largest extent, which sets the radius of exact
// searches in a split grid; rho_max = 0 means cell side >= reach, so the 27
// surrounding cells hold every possible partner.
struct Grid {
  int nc[3];
  int ncell;        // cells of one layer
  double inv_h[3];  // nc / L, for cell assignment only
  double L[3];
  double halfL[3];  // 0.5 * L, the minimum-image threshold
  double h[3];      // L / nc, cell side
  int layer2;       // first cell of the second layer (0: none)
  int walls;        // bit k: reflective walls at 0 and L on axis k (else periodic)
  double rho_max;
  double inv_row;    // 1 / nc0 and 1 / (nc0 nc1): cell coordinates without division
  double inv_layer;
  double sL[3];      // periodic image shift: L on a periodic axis, 0 on a wall axis
};

// Coordinates of cell number c of one layer (c < 2^26, nc0 nc1 <= 2^20)
// without integer division: (c + 0.5) inv is within 2^-26 of the exact
// quotient, whose fractional part is at least 0.5 / divisor >= 2^-21 from an
// integer, so truncating it gives the exact floor.
__device__ __forceinline__ void cell_xyz(const Grid &G, int c, int &cx, int &cy, int &cz) {
  cz = (int)(((double)c + 0.5) * G.inv_layer);
  const int rem = c - cz * (G.nc[0] * G.nc[1]);
  cy = (int)(((double)rem + 0.5) * G.inv_row);
  cx = rem - cy * G.nc[0];
}

// Extent of a sphere over a step, r + |v| dt: two spheres can touch within the
// step only if their separation is at most the sum of their extents.  Written
// once so every kernel classifies a sphere identically.
__device__ __forceinline__ double extent(double r, double vx, double vy, double vz, double dt) {
  return r + __builtin_sqrt((vx * vx + vy * vy) + vz * vz) * dt;
}

// Range-free histogram of positive doubles: the top 16 bits of the binary64
// pattern (11 exponent bits, 4 fraction bits) over exponents 2^-64 .. 2^63,
// 16 bins per octave (bin width at most 1/16 of its lower edge).
constexpr int RHO_BINS = 2048;
__device__ __forceinline__ int rho_bin(double v) {
  const long long b = __double_as_longlong(v) >> 48;  // v > 0: exponent and 4 fraction bits
  const long long k = b - (long long)((1023 - 64) << 4);
  return k < 0 ? 0 : (k >= RHO_BINS ? RHO_BINS - 1 : (int)k);
}

// FP32 copy of a home sphere's record for the pair filter, staged in LDS by
// the detect kernel: position relative to the centre of the home cell, radius,
// velocity (32 B).
struct alignas(16) Rec32 {
  float x, y, z, r;
  float vx, vy, vz, pad;
};

// Values the reach kernel reduces (non-negative doubles compared as bit patterns).
struct ReachOut {
  unsigned long long v2max;  // max over spheres of (vx^2 + vy^2) + vz^2
  unsigned long long rmax;
  unsigned long long rmin;   // initialised to the bits of +inf
  unsigned long long rhomax; // max extent r + |v| dt
  unsigned int bad;          // bit 0: non-finite / r <= 0 / m <= 0; bit 1: position outside [0, L)
  unsigned int maxcell;      // filled by the scan
  unsigned int hist[RHO_BINS];  // extents by rho_bin
};

// One workgroup's share of the reach pass: the bits of its maxima (of
// non-negative doubles, so they order as the values), of its smallest radius
// (+inf if none) and its validity bits.
constexpr int REACH_BLOCKS = 1024;
struct ReachPart {
  unsigned long long v2max, rmax, rmin, rhomax;
  unsigned int bad, pad;
};
__host__ __device__ inline ReachPart reach_merge(const ReachPart &a, const ReachPart &b) {
  return ReachPart{a.v2max > b.v2max ? a.v2max : b.v2max, a.rmax > b.rmax ? a.rmax : b.rmax,
                   a.rmin < b.rmin ? a.rmin : b.rmin, a.rhomax > b.rhomax ? a.rhomax : b.rhomax,
                   a.bad | b.bad, 0u};
}

// The grid of the literal order's space-filling curve: nc cells of side h =
// L / nc per axis (nc <= 2048), independent of the pair-test grid.
struct CurveGrid {
  int nc[3];
  double h[3];
};

// Per-sweep counters the host reads back.  Sums are spread over NSHARD
// counters on separate 128-B lines (one atomic per workgroup on shard
// blockIdx % NSHARD), so no single address takes an atomic per wave.
constexpr int NSHARD = 64;
struct alignas(128) CounterShard {
  unsigned long long pairs;     // pairs resolved this sweep
  unsigned long long contacts;  // contacts found (each counted from both spheres)
  unsigned long long recheck;   // FP32 filter survivors rechecked in FP64 (counted per wave)
  unsigned long long tests;     // pair tests of the large-extent search
  unsigned long long pad[12];
};
struct SweepCounters {
  CounterShard shard[NSHARD];
  unsigned int n_overflow;  // spheres with more contacts than slots (list length)
  unsigned int pad[31];
};

// ---------------------------------------------------------------- the rule

// Contact time of a pair from its minimum-image separation d = x_j - x_i and
// relative velocity u = v_j - v_i (rule 1 of pcol.h; eq. detect1/detect2).
__device__ __forceinline__ bool contact_time(double d0, double d1, double d2, double u0, double u1,
                                             double u2, double s, double dt, double &t) {
  const double a = (u0 * u0 + u1 * u1) + u2 * u2;
  const double b = (d0 * u0 + d1 * u1) + d2 * u2;
  const double c = ((d0 * d0 + d1 * d1) + d2 * d2) - s * s;
  if (!(a > 0.0) || !(b < 0.0) || !(c > 0.0)) return false;
  const double D = b * b - a * c;
  if (!(D >= 0.0)) return false;
  t = c / (-b + __builtin_sqrt(D));
  return t <= dt;
}

// Minimum-image separation along one axis (rule 1).
__device__ __forceinline__ double wrap_sep(double d, double L, double halfL) {
  if (d > halfL) {
    d = d - L;
  } else if (d < -halfL) {
    d = d + L;
  }
  return d;
}

// Final coordinate back into [0, L) (rule 5).
__device__ __forceinline__ double wrap_pos(double p, double L) {
  if (p >= L) {
    p = p - L;
  } else if (p < 0.0) {
    p = p + L;
  }
  if (p >= L) p = 0.0;
  return p;
}

// Time of flight of a centre at x with velocity v until it reaches a wall
// plane (x_k = 0 or L_k on a wall axis), +inf if it moves along no wall axis
// (Sec. "Particle Collisions": a collision counts only before an intersection
// with a domain boundary).
__device__ __forceinline__ double time_to_wall(double x0, double x1, double x2, double v0,
                                               double v1, double v2, const Grid &G) {
  const double x[3] = {x0, x1, x2}, v[3] = {v0, v1, v2};
  double tw = __longlong_as_double(0x7ff0000000000000LL);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (!((G.walls >> k) & 1)) continue;
    double t;
    if (v[k] > 0.0)
      t = (G.L[k] - x[k]) / v[k];
    else if (v[k] < 0.0)
      t = -x[k] / v[k];
    else
      continue;
    tw = t < tw ? t : tw;
  }
  return tw;
}

// Contact at time t of spheres (xa, va) and (xb, vb) allowed by the walls:
// no later than either centre's time of flight to a wall.
__device__ __forceinline__ bool before_walls(double xa0, double xa1, double xa2, double va0,
                                             double va1, double va2, double xb0, double xb1,
                                             double xb2, double vb0, double vb1, double vb2,
                                             const Grid &G, double t) {
  return G.walls == 0 || (t <= time_to_wall(xa0, xa1, xa2, va0, va1, va2, G) &&
                          t <= time_to_wall(xb0, xb1, xb2, vb0, vb1, vb2, G));
}

// Exact contact time of two records with the canonical minimum image (none
// across a wall: halfL is +inf there).  The detect kernels record every such
// contact; the wall condition is applied where partners are chosen
// (k_slot_min, and pair_time_walls in the exact search).
__device__ __forceinline__ bool pair_time(const Rec &a, const Rec &b, const Grid &G, double dt,
                                          double &t) {
  const double d0 = wrap_sep(b.x - a.x, G.L[0], G.halfL[0]);
  const double d1 = wrap_sep(b.y - a.y, G.L[1], G.halfL[1]);
  const double d2 = wrap_sep(b.z - a.z, G.L[2], G.halfL[2]);
  return contact_time(d0, d1, d2, b.vx - a.vx, b.vy - a.vy, b.vz - a.vz, a.r + b.r, dt, t);
}

// pair_time, valid only before either sphere reaches a wall
__device__ __forceinline__ bool pair_time_walls(const Rec &a, const Rec &b, const Grid &G,
                                                double dt, double &t) {
  return pair_time(a, b, G, dt, t) &&
         before_walls(a.x, a.y, a.z, a.vx, a.vy, a.vz, b.x, b.y, b.z, b.vx, b.vy, b.vz, G, t);
}

// End of a flight along axis k, p the unconstrained coordinate: wrapped on a
// periodic axis; on a wall axis reflected at the plane crossed (a perfectly
// reflective wall, Sec. "Intersection of Particles with Solid Walls": the
// velocity component v changes sign), at most one plane per step; a coordinate
// that lands on L itself becomes the largest double below L.
__device__ __forceinline__ double fly_axis(double p, double L, bool wall, double &v) {
  if (!wall) return wrap_pos(p, L);
  if (p >= L) {
    p = L - (p - L);
    v = -v;
  } else if (p < 0.0) {
    p = -p;
    v = -v;
  }
  if (p >= L) p = nextafter(L, 0.0);
  return p;
}

// Post-collision state of sphere `a` colliding with `b` at time t (rule 4,
// Sec. "Inter-Particle Collisions" with friction 0, eq. update_vel/update_rho).
// Bitwise independent of which of the two is `a`.
__device__ __forceinline__ void resolve_one(const Rec &a, const Rec &b, double ma, double mb,
                                            const Grid &G, double t, double dt, double e,
                                            double out_x[3], double out_v[3]) {
  const double d0 = wrap_sep(b.x - a.x, G.L[0], G.halfL[0]);
  const double d1 = wrap_sep(b.y - a.y, G.L[1], G.halfL[1]);
  const double d2 = wrap_sep(b.z - a.z, G.L[2], G.halfL[2]);
  const double u0 = b.vx - a.vx, u1 = b.vy - a.vy, u2 = b.vz - a.vz;
  const double s = a.r + b.r;
  const double n0 = (d0 + t * u0) / s;
  const double n1 = (d1 + t * u1) / s;
  const double n2 = (d2 + t * u2) / s;
  const double g = (u0 * n0 + u1 * n1) + u2 * n2;
  const double mr = (ma * mb) / (ma + mb);
  const double J = (mr * (1.0 + e)) * g;
  const double ai = J / ma;
  out_v[0] = a.vx + ai * n0;
  out_v[1] = a.vy + ai * n1;
  out_v[2] = a.vz + ai * n2;
  const double rest = dt - t;
  out_x[0] = fly_axis((a.x + t * a.vx) + rest * out_v[0], G.L[0], G.walls & 1, out_v[0]);
  out_x[1] = fly_axis((a.y + t * a.vy) + rest * out_v[1], G.L[1], G.walls & 2, out_v[1]);
  out_x[2] = fly_axis((a.z + t * a.vz) + rest * out_v[2], G.L[2], G.walls & 4, out_v[2]);
}

// Angular velocities (caller order, updated in place for collided spheres) and
// the Coulomb friction coefficient of a step with spin; wx == nullptr: none.
struct Spin {
  double *wx, *wy, *wz;
  double mu;
};

// Post-collision state of sphere `a` colliding with `b` at time t with Coulomb
// friction mu and spins wa, wb (Sec. "Inter-Particle Collisions": impulse
// J = J_n n + J_t t_p, J_t = max(mu J_n, -(2/7)(1+e) m_r |v_rt|), jump
// relations of momentum and angular momentum; solid-sphere inertia m d^2 / 10,
// Sec. "Dispersed Phase").  The contact-point velocity is evaluated as
// v_r + (r_a w_a + r_b w_b) x n, so b's evaluation is the exact negation of a's
// and the two sides agree bitwise; with J_t = 0 the tangential terms are left
// out (then the velocity equals resolve_one's and the spin is unchanged).
__device__ __forceinline__ void resolve_one_spin(const Rec &a, const Rec &b, double ma, double mb,
                                                 const double wa[3], const double wb[3],
                                                 const Grid &G, double t, double dt, double e,
                                                 double mu, double out_x[3], double out_v[3],
                                                 double out_w[3]) {
  const double d0 = wrap_sep(b.x - a.x, G.L[0], G.halfL[0]);
  const double d1 = wrap_sep(b.y - a.y, G.L[1], G.halfL[1]);
  const double d2 = wrap_sep(b.z - a.z, G.L[2], G.halfL[2]);
  const double u[3] = {b.vx - a.vx, b.vy - a.vy, b.vz - a.vz};
  const double s = a.r + b.r;
  const double n[3] = {(d0 + t * u[0]) / s, (d1 + t * u[1]) / s, (d2 + t * u[2]) / s};
  const double g = (u[0] * n[0] + u[1] * n[1]) + u[2] * n[2];
  const double mr = (ma * mb) / (ma + mb);
  const double Jn = (mr * (1.0 + e)) * g;
  double S[3];
  for (int k = 0; k < 3; ++k) S[k] = a.r * wa[k] + b.r * wb[k];
  const double Sxn[3] = {S[1] * n[2] - S[2] * n[1], S[2] * n[0] - S[0] * n[2],
                         S[0] * n[1] - S[1] * n[0]};
  double vc[3];
  for (int k = 0; k < 3; ++k) vc[k] = -u[k] + Sxn[k];
  const double vcn = (vc[0] * n[0] + vc[1] * n[1]) + vc[2] * n[2];
  double vrt[3];
  for (int k = 0; k < 3; ++k) vrt[k] = vc[k] - vcn * n[k];
  const double vt = __builtin_sqrt((vrt[0] * vrt[0] + vrt[1] * vrt[1]) + vrt[2] * vrt[2]);
  double Jt = 0.0, tp[3] = {0.0, 0.0, 0.0};
  if (vt > 0.0) {
    for (int k = 0; k < 3; ++k) tp[k] = vrt[k] / vt;
    const double slide = mu * Jn;
    const double stick = -((((2.0 / 7.0) * (1.0 + e)) * mr) * vt);
    Jt = slide > stick ? slide : stick;
  }
  const double an = Jn / ma, at = Jt / ma;
  const double va[3] = {a.vx, a.vy, a.vz}, xa[3] = {a.x, a.y, a.z};
  const double rest = dt - t;
  for (int k = 0; k < 3; ++k) {
    double v = va[k] + an * n[k];
    if (Jt != 0.0) v = v + at * tp[k];
    double vk = v;  // reflected on a wall axis (the spin is unchanged by an elastic wall)
    out_x[k] = fly_axis((xa[k] + t * va[k]) + rest * v, G.L[k], (G.walls >> k) & 1, vk);
    out_v[k] = vk;
    out_w[k] = wa[k];
  }
  if (Jt != 0.0) {
    const double da = 2.0 * a.r;
    const double I = (ma * (da * da)) / 10.0;
    const double K = (a.r * Jt) / I;
    const double nxt[3] = {n[1] * tp[2] - n[2] * tp[1], n[2] * tp[0] - n[0] * tp[2],
                           n[0] * tp[1] - n[1] * tp[0]};
    for (int k = 0; k < 3; ++k) out_w[k] = wa[k] + K * nxt[k];
  }
}

__device__ __forceinline__ int cell_coord(double x, double inv_h, int nc) {
  int c = (int)(x * inv_h);
  c = c < 0 ? 0 : c;
  return c > nc - 1 ? nc - 1 : c;
}

// ---------------------------------------------------------------- launches

struct Particles {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz;
  const double *r, *m;
  const double *wx = nullptr, *wy = nullptr, *wz = nullptr;  // spins, validated when given
};

// gradient with respect to a step's positions and velocities (SoA)
struct StateGrad {
  double *x, *y, *z, *vx, *vy, *vz;
};

// Device tables of the batched form: one grid per box, boxes' cells numbered
// consecutively (cell_base), the box of every sphere, and status flags that
// let every kernel of a captured step skip its work.
enum { FLAG_DONE = 0, FLAG_ERR = 1, FLAG_SWEEPS = 2, FLAG_UNFINISHED = 3 };
enum : unsigned int { ERR_INVALID = 1u, ERR_REPLAN = 2u, ERR_BOX = 4u };
// A box's maxima during the batched reach pass (bits of non-negative doubles)
// and its validity bits; zero between passes.
struct BoxMax {
  unsigned long long v2, rm;
  unsigned int bad, pad;
};
// Spheres per workgroup of the batched reach pass (a box spans one or more).
constexpr int BREACH_CHUNK = 4096;

struct BatchDev {
  const Grid *gtab;       // [nbox]
  const int *cell_base;   // [nbox + 1]
  const int *box_of;      // caller order: box of each sphere
  const int64_t *box_off; // [nbox + 1] sphere ranges (caller order)
  double *breach;         // [nbox] reach found by the last step
  unsigned int *flags;    // FLAG_* words
  int nbox;
  int nchunk;             // chunks of the reach pass: box chunk_box[k], spheres from chunk_lo[k]
  const int *chunk_box;
  const int64_t *chunk_lo;
  BoxMax *bmax;           // [nbox]
};

// Pair tests and filter survivors of one workgroup of the k_detect_half kernels.
struct CellCount {
  unsigned long long tests, recheck;
};

// Everything the sweep-1 detect needs.
struct DetectArgs {
  const Rec *rec;
  const int *start;   // ncell + 1
  int *cnt;           // per sorted sphere: contacts found
  double *slot_t;     // [n * K]
  int *slot_j;        // [n * K]
  SweepCounters *ctr;
  int n;              // spheres (slot arrays are k-major: slot[k * n + i])
  Grid G;
  double dt;
  double dt2;         // 2 dt (1 + 2^-20): step bound of the FP64 filter
  double tol;         // binary32 filter: unused; kept for the FMA form's bound
  double tol64;       // binary64 Gram filter tolerance (see gram64_tolerance)
  double tol_wide;    // the same for pairs with a sphere above the split extent (full reach)
  double rho_c;       // split extent (first-layer spheres have extent <= rho_c)
  int K;
  int fp32;           // FP32 filter + FP64 recheck
  float kband;        // FP32 filter: contact distance inflated to s * kband
  float dt2f;         // FP32 filter: 2 dt (1 + 2^-12)
  CellCount *cellc;   // per workgroup of the one-box detect kernels (G.ncell entries)
  int cpw;            // binary64 filter: home cells per workgroup (1: one cell per wave)
};

hipError_t launch_fill_u32(hipStream_t s, unsigned int *p, unsigned int v, int64_t n);
hipError_t launch_fill_u8(hipStream_t s, uint8_t *p, uint8_t v, int64_t n);
hipError_t launch_fill_f64(hipStream_t s, double *p, double v, int64_t n);
hipError_t launch_fill_i32(hipStream_t s, int *p, int v, int64_t n);
// hist_shift: the extent histogram covers the spheres whose index is a multiple
// of 2^hist_shift (the maxima and the validity cover all).  parts and phist are
// scratch of REACH_BLOCKS partial results and REACH_BLOCKS * RHO_BINS counts;
// out->hist must be zero and out's other fields are overwritten.  G given: the
// pass also bins the spheres on G with split extent rho_c into cid, slot and
// count (zero on entry), as launch_cell_hist does.
hipError_t launch_reach(hipStream_t s, const Particles &P, const double L[3], double dt,
                        int hist_shift, ReachOut *out, ReachPart *parts, unsigned int *phist,
                        const Grid *G = nullptr, double rho_c = 0.0, int *cid = nullptr,
                        int *slot = nullptr, int *count = nullptr);
hipError_t launch_cell_hist(hipStream_t s, const Particles &P, const Grid &G, double dt,
                            double rho_c, int *cid, int *slot, int *count);
// the spheres of the second layer, sorted positions [*first_dev, n)
hipError_t launch_detect_wide(hipStream_t s, const DetectArgs &A, const int *first_dev, int n);
hipError_t launch_scan(hipStream_t s, const int *count, int ncell, int *start, int *blocksum,
                       ReachOut *out);
hipError_t launch_scatter(hipStream_t s, const Particles &P, const int *cid, const int *slot,
                          const int *start, Rec *rec, int *rank, const BatchDev *B);
hipError_t launch_detect_half(hipStream_t s, const DetectArgs &A);
// workgroups of launch_detect_half, each writing one CellCount
int detect_half_blocks(const DetectArgs &A);
// adds the per-cell counts of launch_detect_half to the counter shards of ctr
hipError_t launch_cell_counts(hipStream_t s, const CellCount *c, int n, SweepCounters *ctr);
hipError_t launch_slot_min(hipStream_t s, int n, int first, const int *cnt, const double *slot_t,
                           const int *slot_j, int K, uint8_t *status, const Rec *rec, int *key_j,
                           double *key_t, int *ovf_list, SweepCounters *ctr,
                           const unsigned int *flags, const int *list = nullptr, int nlist = 0,
                           const Grid *G = nullptr,  // G: walls of the single box (none: periodic)
                           const unsigned long long *crank = nullptr);  // literal order's ranks
hipError_t launch_gather_exact(hipStream_t s, const int *list, int nlist, const unsigned int *nlist_dev,
                               int select, const Rec *rec, const int *start, const Grid &G,
                               double dt, uint8_t *status, int *key_j, double *key_t,
                               const BatchDev *B, const unsigned long long *crank = nullptr);
hipError_t launch_curve_rank(hipStream_t s, const Rec *rec, int n, const CurveGrid &C,
                             unsigned long long *crank);
// spin (nullable): friction and spins (the pair's sphere of smaller sorted index
// resolves both sides and writes both spins in place)
hipError_t launch_resolve_sweep(hipStream_t s, int n, const Rec *rec, const Grid &G, double dt,
                                double e, const double *mass, const int *key_j,
                                const double *key_t, uint8_t *status, OutRec *out,
                                SweepCounters *ctr,
                                const BatchDev *B,
                                const int *list = nullptr, int nlist = 0,
                                const Spin *spin = nullptr);
// list (read back from off[(n + 255) / 256] entries) of the ACTIVE or
// DIRTY spheres; count and off need (n + 255) / 256 + 1 entries, blocksum
// ((n + 255) / 256) / 4096 + 2
hipError_t launch_keep_list(hipStream_t s, const uint8_t *status, int n, int *count, int *off,
                            int *blocksum, ReachOut *scratch_out, int *list);
hipError_t launch_finish(hipStream_t s, const Particles &P, const int *rank, const OutRec *out,
                         const uint8_t *status, int *partner, double *tcoll, double dt,
                         const Grid &G, const BatchDev *B);
hipError_t launch_fill_box_of(hipStream_t s, int nbox, const int64_t *box_off, int *box_of);
// count given (zero on entry): the pass also takes every sphere's global cell
// (box's first cell + local cell on its planned grid) and its slot in that cell
// into cid, slot and count
hipError_t launch_breach(hipStream_t s, const Particles &P, const BatchDev &B, double dt,
                         int check_plan, int *cid = nullptr, int *slot = nullptr,
                         int *count = nullptr);
// cpw consecutive global cells per workgroup (one wave) over total_cells
hipError_t launch_detect_batched(hipStream_t s, const DetectArgs &A, const BatchDev &B,
                                 int total_cells, int cpw);
hipError_t launch_sweep_check(hipStream_t s, SweepCounters *ctr, unsigned int *flags,
                              unsigned long long *totals, int last);
hipError_t launch_advance(hipStream_t s, const Particles &P, const int *partner, double dt,
                          const double L[3]);
hipError_t launch_status_from_active(hipStream_t s, const uint8_t *active, const Rec *rec, int n,
                                     uint8_t *status);
hipError_t launch_export_keys(hipStream_t s, int n, const Rec *rec, const int *key_j,
                              const double *key_t, const uint8_t *status, uint64_t *key_out,
                              double *tmin_out);
hipError_t launch_step_backward(hipStream_t s, const Particles &P, const Grid &G, double dt,
                                double e, const int *partner, const double *tcoll,
                                const StateGrad &gout, const StateGrad &gin, double *ebuf,
                                double *ge);
// Deposition of per-sphere sources onto the corner nodes of a periodic
// Cartesian grid: positions x, y, z (n), sources a[q * n + i] (comp <= 8),
// nc cells of side h = L / nc per axis, out[node * comp + q] (nnode nodes,
// one per element).  Scratch: eid, slot (n each), cnt (nnode, zeroed before the
// count), start (nnode + 1), rec (n records of deposit_record_bytes(comp)).
struct DepositArgs {
  const double *x, *y, *z, *a;
  int64_t n;
  int comp;
  int nc[3];
  double L[3], h[3];
  int64_t nnode;
  double *out;
  int *eid, *slot, *cnt, *start;
  void *rec;
};
int64_t deposit_record_bytes(int comp);
// element and slot of every sphere (cnt must be zero); positions outside
// [0, L) or not finite set bit 0 of *flag and are skipped
hipError_t launch_deposit_count(hipStream_t s, const DepositArgs &D, unsigned int *flag);
// after the scan of cnt into start: scatter, then element corner sums and node
// sums over tiles of nodes
hipError_t launch_deposit(hipStream_t s, const DepositArgs &D);
hipError_t launch_resolve_public(hipStream_t s, int n, const Rec *rec, const int *rank,
                                 const Grid &G, double dt, double e, const uint64_t *key,
                                 const Particles &P, uint8_t *active, int *partner, double *tcoll,
                                 long long *npairs);

}  // namespace pcol
