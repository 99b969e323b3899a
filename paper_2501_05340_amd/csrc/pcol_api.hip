// C-ABI layer of the pcol library: argument checks, the context and its
// device scratch, the grid choice, and the sweep driver of pcol_step.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "../../include/pcol.h"
#include "pcol_internal.h"

using namespace pcol;

struct pcol_ctx {
  int64_t n_max = 0;
  hipStream_t stream = nullptr;
  pcol_opts opts{};
  std::string err;
  int K = 12;

  // cell-sorted state of the last pcol_bin
  Rec *rec = nullptr;
  Rec32 *rec32 = nullptr;  // FP32 filter records (fp32_filter only)
  int *perm = nullptr;  // sorted position -> caller index
  int *rank = nullptr;  // caller index -> sorted position
  int *cid = nullptr;
  int *slot = nullptr;
  int *count = nullptr;
  int *start = nullptr;
  int *blocksum = nullptr;
  int64_t cell_cap = 0;

  // sweep state
  int *cnt = nullptr;
  double *slot_t = nullptr;
  int *slot_j = nullptr;
  int *key_j = nullptr;
  double *key_t = nullptr;
  uint8_t *status = nullptr;
  int *ovf = nullptr;
  OutRec *out = nullptr;
  int *partner_tmp = nullptr;
  double *tcoll_tmp = nullptr;
  ReachOut *reach_d = nullptr;
  SweepCounters *ctr_d = nullptr;
  unsigned long long *tests_d = nullptr;
  ReachOut *reach_h = nullptr;
  SweepCounters *ctr_h = nullptr;
  unsigned long long *tests_h = nullptr;
  hipEvent_t ev[8] = {};

  bool binned = false;
  int64_t binned_n = -1;
  const double *binned_x = nullptr;
  Grid G{};
  double reach = 0.0;
  double vmax = 0.0, rmin = 0.0, rmax = 0.0;
  double band = 0.0;   // FP32 filter band in use (relative to r_i + r_j)
  double h[3] = {0, 0, 0};
  int maxcell = 0;
  bool small = false;  // some axis has fewer than 3 cells
  bool detect_timed = false;
};

namespace {

pcol_status fail(pcol_ctx *c, pcol_status st, const char *what) {
  if (c) c->err = what;
  return st;
}

pcol_status hip_fail(pcol_ctx *c, hipError_t e, const char *where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return PCOL_E_HIP;
}

#define PCOL_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, (count ? count : 1) * sizeof(T));
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

pcol_status check_common(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt) {
  if (!ctx) return PCOL_E_INVALID;
  if (!p || !box) return fail(ctx, PCOL_E_INVALID, "null particles or box");
  if (p->n < 0 || p->n > ctx->n_max) return fail(ctx, PCOL_E_INVALID, "n outside [0, n_max]");
  if (p->n > 0 && (!p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->r || !p->m))
    return fail(ctx, PCOL_E_INVALID, "null particle array");
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(box->len[a])) return fail(ctx, PCOL_E_INVALID, "box side not finite positive");
  if (!finite_pos(dt)) return fail(ctx, PCOL_E_INVALID, "dt not finite positive");
  return PCOL_OK;
}

Particles to_dev(const pcol_particles *p) {
  Particles P;
  P.n = p->n;
  P.x = p->x;
  P.y = p->y;
  P.z = p->z;
  P.vx = p->vx;
  P.vy = p->vy;
  P.vz = p->vz;
  P.r = p->r;
  P.m = p->m;
  return P;
}

double ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

}  // namespace

extern "C" {

void pcol_default_opts(pcol_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->cell_mult = 1.0;
  o->max_sweeps = 0;
  o->home_cells = 0;
  o->contact_slots = 12;
  o->fp32_filter = 0;
  o->band_rel = 1e-4;
  o->timing = 0;
}

const char *pcol_last_error(const pcol_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

pcol_status pcol_set_stream(pcol_ctx *ctx, void *hip_stream) {
  if (!ctx) return PCOL_E_INVALID;
  ctx->stream = (hipStream_t)hip_stream;
  return PCOL_OK;
}

void pcol_destroy(pcol_ctx *ctx) {
  if (!ctx) return;
  void *dev[] = {ctx->rec,    ctx->rec32,  ctx->perm,   ctx->rank,   ctx->cid,         ctx->slot,
                 ctx->count,  ctx->start,  ctx->blocksum, ctx->cnt,      ctx->slot_t,
                 ctx->slot_j, ctx->key_j,  ctx->key_t,  ctx->status,      ctx->out,
                 ctx->ovf,    ctx->partner_tmp, ctx->tcoll_tmp,
                 ctx->reach_d, ctx->ctr_d, ctx->tests_d};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  if (ctx->reach_h) (void)hipHostFree(ctx->reach_h);
  if (ctx->ctr_h) (void)hipHostFree(ctx->ctr_h);
  if (ctx->tests_h) (void)hipHostFree(ctx->tests_h);
  for (hipEvent_t &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

pcol_status pcol_create(pcol_ctx **out, int64_t n_max, void *hip_stream, const pcol_opts *opts) {
  if (!out) return PCOL_E_INVALID;
  *out = nullptr;
  if (n_max < 0 || n_max > 0x7fffffffLL) return PCOL_E_INVALID;
  pcol_ctx *ctx = new (std::nothrow) pcol_ctx();
  if (!ctx) return PCOL_E_NOMEM;
  pcol_default_opts(&ctx->opts);
  if (opts) ctx->opts = *opts;
  if (!(ctx->opts.cell_mult >= 1.0) || !isfinite(ctx->opts.cell_mult) ||
      ctx->opts.max_sweeps < 0 || ctx->opts.contact_slots < 0 || ctx->opts.contact_slots > 64 ||
      !(ctx->opts.band_rel >= 0.0)) {
    delete ctx;
    return PCOL_E_INVALID;
  }
  ctx->K = ctx->opts.contact_slots > 0 ? ctx->opts.contact_slots : 12;
  ctx->n_max = n_max;
  ctx->stream = (hipStream_t)hip_stream;
  const size_t n = (size_t)n_max;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  A(dalloc(&ctx->rec, n));
  if (ctx->opts.fp32_filter) A(dalloc(&ctx->rec32, n));
  A(dalloc(&ctx->perm, n));
  A(dalloc(&ctx->rank, n));
  A(dalloc(&ctx->cid, n));
  A(dalloc(&ctx->slot, n));
  A(dalloc(&ctx->cnt, n));
  A(dalloc(&ctx->slot_t, n * (size_t)ctx->K));
  A(dalloc(&ctx->slot_j, n * (size_t)ctx->K));
  A(dalloc(&ctx->key_j, n));
  A(dalloc(&ctx->key_t, n));
  A(dalloc(&ctx->status, n));
  A(dalloc(&ctx->out, n));
  A(dalloc(&ctx->ovf, n));
  A(dalloc(&ctx->partner_tmp, n));
  A(dalloc(&ctx->tcoll_tmp, n));
  A(dalloc(&ctx->reach_d, 1));
  A(dalloc(&ctx->ctr_d, 1));
  A(dalloc(&ctx->tests_d, 1));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->reach_h, sizeof(ReachOut));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->ctr_h, sizeof(SweepCounters));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->tests_h, sizeof(unsigned long long));
  for (hipEvent_t &ev : ctx->ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e != hipSuccess) {
    pcol_destroy(ctx);
    return e == hipErrorOutOfMemory ? PCOL_E_NOMEM : PCOL_E_HIP;
  }
  *out = ctx;
  return PCOL_OK;
}

pcol_status pcol_bin(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  ctx->binned = false;
  const Particles P = to_dev(p);
  hipStream_t s = ctx->stream;
  // a1: reach and data validity (one read-back)
  PCOL_HIP(hipMemsetAsync(ctx->reach_d, 0, sizeof(ReachOut), s));
  PCOL_HIP(launch_fill_u32(s, (unsigned int *)&ctx->reach_d->rmin, 0u, 1));
  PCOL_HIP(launch_fill_u32(s, (unsigned int *)&ctx->reach_d->rmin + 1, 0x7ff00000u, 1));
  PCOL_HIP(launch_reach(s, P, box->len, ctx->reach_d));
  PCOL_HIP(hipMemcpyAsync(ctx->reach_h, ctx->reach_d, sizeof(ReachOut), hipMemcpyDeviceToHost, s));
  PCOL_HIP(hipStreamSynchronize(s));
  const ReachOut ro = *ctx->reach_h;
  if (ro.bad & 1u) return fail(ctx, PCOL_E_INVALID, "non-finite value, r <= 0 or m <= 0");
  if (ro.bad & 2u) return fail(ctx, PCOL_E_INVALID, "position outside [0, L)");
  double v2, rmax, rmin;
  memcpy(&v2, &ro.v2max, sizeof(double));
  memcpy(&rmax, &ro.rmax, sizeof(double));
  memcpy(&rmin, &ro.rmin, sizeof(double));
  const double reach = 2.0 * rmax + 2.0 * sqrt(v2) * dt;
  for (int a = 0; a < 3; ++a)
    if (!(box->len[a] > 2.0 * reach))
      return fail(ctx, PCOL_E_BOX, "box side <= 2 * reach: minimum image not unique");
  // grid: cell side >= reach * cell_mult, at most 2^27 cells
  Grid G{};
  double cell = reach * ctx->opts.cell_mult;
  if (!(cell > 0.0)) cell = box->len[0];  // no motion and no size: one cell
  for (;;) {
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
      double q = floor(box->len[a] / (cell * (1.0 + 1e-9)));
      if (!(q >= 1.0)) q = 1.0;
      if (q > 1024.0) q = 1024.0;
      G.nc[a] = (int)q;
      ncell *= G.nc[a];
    }
    if (ncell <= (1 << 27)) {
      G.ncell = (int)ncell;
      break;
    }
    cell *= 1.25;
  }
  ctx->small = false;
  for (int a = 0; a < 3; ++a) {
    G.L[a] = box->len[a];
    G.halfL[a] = 0.5 * box->len[a];
    G.inv_h[a] = (double)G.nc[a] / box->len[a];
    G.h[a] = box->len[a] / G.nc[a];
    ctx->h[a] = G.h[a];
    if (G.nc[a] < 3) ctx->small = true;
  }
  if ((int64_t)G.ncell + 2 > ctx->cell_cap) {
    if (ctx->count) (void)hipFree(ctx->count);
    if (ctx->start) (void)hipFree(ctx->start);
    if (ctx->blocksum) (void)hipFree(ctx->blocksum);
    ctx->count = ctx->start = ctx->blocksum = nullptr;
    ctx->cell_cap = 0;
    const int64_t cap = (int64_t)G.ncell + 2;
    hipError_t e = dalloc(&ctx->count, (size_t)cap);
    if (e == hipSuccess) e = dalloc(&ctx->start, (size_t)cap + 1);
    if (e == hipSuccess) e = dalloc(&ctx->blocksum, (size_t)(cap / 4096 + 2));
    if (e != hipSuccess) return fail(ctx, PCOL_E_NOMEM, "cell arrays");
    ctx->cell_cap = cap;
  }
  // a2-a4: counting sort into cell-sorted records
  PCOL_HIP(launch_fill_i32(s, ctx->count, 0, G.ncell));
  PCOL_HIP(launch_cell_hist(s, P, G, ctx->cid, ctx->slot, ctx->count));
  PCOL_HIP(launch_scan(s, ctx->count, G.ncell, ctx->start, ctx->blocksum, ctx->reach_d));
  PCOL_HIP(launch_scatter(s, P, G, ctx->cid, ctx->slot, ctx->start, ctx->rec,
                          ctx->opts.fp32_filter ? ctx->rec32 : nullptr, ctx->perm, ctx->rank));
  PCOL_HIP(hipMemcpyAsync(ctx->reach_h, ctx->reach_d, sizeof(ReachOut), hipMemcpyDeviceToHost, s));
  PCOL_HIP(hipStreamSynchronize(s));
  ctx->maxcell = (int)ctx->reach_h->maxcell;
  ctx->G = G;
  ctx->reach = reach;
  ctx->vmax = sqrt(v2);
  ctx->rmin = rmin;
  ctx->rmax = rmax;
  ctx->binned = true;
  ctx->binned_n = p->n;
  ctx->binned_x = p->x;
  return PCOL_OK;
}

static pcol_status check_binned(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box) {
  if (!ctx->binned || ctx->binned_n != p->n)
    return fail(ctx, PCOL_E_STATE, "pcol_bin must run first on the same particle set");
  for (int a = 0; a < 3; ++a)
    if (box->len[a] != ctx->G.L[a]) return fail(ctx, PCOL_E_STATE, "box differs from pcol_bin");
  return PCOL_OK;
}

// Contact-distance factor of the FP32 filter.  Bounds (unit roundoff u = 2^-24)
// on the FP32 errors of the filter quantities for any pair the binary64 rule
// can keep (|d| <= reach, |u| <= 2 vmax, coordinates within 1.5 h of the home
// cell centre):
//   separation   Dd = (2 h + reach) u       relative velocity  Du = 4 vmax u
//   c' = |d|^2 - (s k)^2:  2 sqrt3 reach Dd + 3 u reach^2 + 6 u (2 rmax k)^2
//   b' dt2f = d.u dt2f:    (sqrt3 (reach Du + 2 vmax Dd) + 6 u reach vmax) 2 dt (1 + 2^-11)
// The inflation (k^2 - 1) s_min^2 >= 2 (k - 1) s_min^2 must cover their sum; k
// is chosen so that it covers twice the sum, and never below 1 + band_rel.
static double fp32_band(const pcol_ctx *ctx, double dt) {  // returns the band
  const double u = 0x1.0p-24;
  double h = ctx->h[0];
  for (int a = 1; a < 3; ++a) h = ctx->h[a] > h ? ctx->h[a] : h;
  const double R = ctx->reach, V = ctx->vmax, smin = 2.0 * ctx->rmin;
  const double k0 = 1.0 + ctx->opts.band_rel + 1e-3;  // generous k for the radius term
  const double Dd = (2.0 * h + R) * u, Du = 4.0 * V * u;
  const double ec = 2.0 * sqrt(3.0) * R * Dd + 3.0 * u * R * R +
                    6.0 * u * (2.0 * ctx->rmax * k0) * (2.0 * ctx->rmax * k0);
  const double eb = (sqrt(3.0) * (R * Du + 2.0 * V * Dd) + 6.0 * u * R * V) * 2.0 * dt *
                    (1.0 + 0x1.0p-11);
  const double need = 2.0 * (ec + eb) / (2.0 * smin * smin);
  return ctx->opts.band_rel > need ? ctx->opts.band_rel : need;
}

// sweep 1: keys of all spheres (all active) into ctx->key_j / key_t (sorted order)
static pcol_status detect_all(pcol_ctx *ctx, double dt) {
  hipStream_t s = ctx->stream;
  const int n = (int)ctx->binned_n;
  if (!ctx->small) {
    DetectArgs A{};
    A.rec = ctx->rec;
    A.start = ctx->start;
    A.cnt = ctx->cnt;
    A.slot_t = ctx->slot_t;
    A.slot_j = ctx->slot_j;
    A.ctr = ctx->ctr_d;
    A.n = n;
    A.G = ctx->G;
    A.dt = dt;
    A.dt2 = 2.0 * dt * (1.0 + 0x1.0p-20);
    {
      // 16 eps (reach^2 + (2 rmax)^2 + reach * 2 vmax * dt2): twice the bound on the
      // differences between the filter's FMA values and the rule's b, c (pair64)
      const double R = ctx->reach, smax = 2.0 * ctx->rmax;
      A.tol = 16.0 * 0x1.0p-53 * (R * R + smax * smax + R * 2.0 * ctx->vmax * A.dt2);
    }
    A.K = ctx->K;
    A.rec32 = ctx->rec32;
    A.fp32 = ctx->opts.fp32_filter;
    // the FP32 filter reads its home records from an LDS copy of the home cell
    // (when the largest cell fits in 20 KB); the FP64 filter reads them through
    // the scalar cache, which measured faster for 64-B records
    A.cap = A.fp32 && ctx->maxcell * (int)sizeof(Rec32) <= 20 * 1024
                ? (ctx->maxcell > 0 ? ctx->maxcell : 1)
                : 0;
    ctx->band = A.fp32 ? fp32_band(ctx, dt) : 0.0;
    // round the factor up so the float never shrinks the inflation
    const double kb = 1.0 + ctx->band;
    A.kband = (float)kb;
    if ((double)A.kband < kb) A.kband = nextafterf(A.kband, 2.0f);
    A.dt2f = (float)(2.0 * dt * (1.0 + 0x1.0p-12));
    PCOL_HIP(launch_fill_i32(s, ctx->cnt, 0, n));
    if (ctx->opts.timing) PCOL_HIP(hipEventRecord(ctx->ev[5], s));
    PCOL_HIP(launch_detect_half(s, A));
    if (ctx->opts.timing) PCOL_HIP(hipEventRecord(ctx->ev[6], s));
    ctx->detect_timed = true;
    PCOL_HIP(launch_slot_min(s, n, 1, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                             ctx->perm, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d));
    PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec, ctx->start,
                                 ctx->G, dt, ctx->status, ctx->perm, ctx->key_j, ctx->key_t));
  } else {
    // fewer than 3 cells on some axis: exact search for every sphere
    PCOL_HIP(launch_gather_exact(s, nullptr, n, nullptr, -1, ctx->rec, ctx->start, ctx->G, dt,
                                 ctx->status, ctx->perm, ctx->key_j, ctx->key_t));
  }
  return PCOL_OK;
}

static void sum_counters(const SweepCounters &c, unsigned long long &pairs,
                         unsigned long long &contacts) {
  pairs = contacts = 0ull;
  for (int k = 0; k < NSHARD; ++k) {
    pairs += c.shard[k].pairs;
    contacts += c.shard[k].contacts;
  }
}

pcol_status pcol_detect(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt,
                        const uint8_t *active, uint64_t *key_out, double *tmin_out) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if ((st = check_binned(ctx, p, box)) != PCOL_OK) return st;
  if (p->n > 0 && !key_out) return fail(ctx, PCOL_E_INVALID, "key_out is null");
  hipStream_t s = ctx->stream;
  const int n = (int)p->n;
  if (n == 0) return PCOL_OK;
  PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
  if (!active) {
    PCOL_HIP(launch_fill_u8(s, ctx->status, ST_ACTIVE, n));
    if ((st = detect_all(ctx, dt)) != PCOL_OK) return st;
  } else {
    PCOL_HIP(launch_status_from_active(s, active, ctx->perm, n, ctx->status));
    PCOL_HIP(launch_fill_i32(s, ctx->key_j, -1, n));
    PCOL_HIP(launch_gather_exact(s, nullptr, n, nullptr, ST_ACTIVE, ctx->rec, ctx->start, ctx->G,
                                 dt, ctx->status, ctx->perm, ctx->key_j, ctx->key_t));
  }
  PCOL_HIP(launch_export_keys(s, n, ctx->perm, ctx->key_j, ctx->key_t, ctx->status, key_out,
                              tmin_out));
  return PCOL_OK;
}

pcol_status pcol_resolve(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                         double e, const uint64_t *key, uint8_t *active, int32_t *partner,
                         double *tcoll, int64_t *n_pairs_dev) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  if ((st = check_binned(ctx, p, box)) != PCOL_OK) return st;
  if (p->n > 0 && (!key || !active)) return fail(ctx, PCOL_E_INVALID, "key or active is null");
  PCOL_HIP(launch_resolve_public(ctx->stream, (int)p->n, ctx->rec, ctx->rank, ctx->G, dt, e, key,
                                 to_dev(p), active, partner, tcoll, (long long *)n_pairs_dev));
  return PCOL_OK;
}

pcol_status pcol_advance(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                         const int32_t *partner) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if (p->n > 0 && !partner) return fail(ctx, PCOL_E_INVALID, "partner is null");
  PCOL_HIP(launch_advance(ctx->stream, to_dev(p), partner, dt, box->len));
  return PCOL_OK;
}

pcol_status pcol_step(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt, double e,
                      int32_t *partner, double *tcoll, pcol_stats *stats) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  hipStream_t s = ctx->stream;
  const bool timing = ctx->opts.timing != 0;
  if (timing) PCOL_HIP(hipEventRecord(ctx->ev[0], s));
  if ((st = pcol_bin(ctx, p, box, dt)) != PCOL_OK) return st;
  if (timing) PCOL_HIP(hipEventRecord(ctx->ev[1], s));
  const int n = (int)p->n;
  int32_t *part = partner ? partner : ctx->partner_tmp;
  double *tc = tcoll ? tcoll : ctx->tcoll_tmp;
  const Particles P = to_dev(p);
  int64_t pairs = 0, sweeps = 0, ovf_total = 0;
  unsigned long long contacts = 0ull, recheck = 0ull;
  double ms_detect = 0.0;
  if (n > 0) {
    PCOL_HIP(launch_fill_u8(s, ctx->status, ST_ACTIVE, n));
    PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
    // sweep 1: every contact within dt, then the earliest partner of each sphere
    ctx->detect_timed = false;
    if ((st = detect_all(ctx, dt)) != PCOL_OK) return st;
    if (timing) PCOL_HIP(hipEventRecord(ctx->ev[2], s));
    for (;;) {
      PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, ctx->key_j, ctx->key_t,
                                    ctx->status, ctx->perm, ctx->out, ctx->ctr_d));
      PCOL_HIP(hipMemcpyAsync(ctx->ctr_h, ctx->ctr_d, sizeof(SweepCounters),
                              hipMemcpyDeviceToHost, s));
      PCOL_HIP(hipStreamSynchronize(s));
      unsigned long long sp, sc;
      sum_counters(*ctx->ctr_h, sp, sc);
      if (sweeps == 0) {
        contacts = sc / 2ull;
        for (int k = 0; k < NSHARD; ++k) recheck += ctx->ctr_h->shard[k].recheck;
      }
      ovf_total += ctx->ctr_h->n_overflow;
      ++sweeps;
      pairs += (int64_t)sp;
      if (sp == 0ull) break;
      if (ctx->opts.max_sweeps > 0 && sweeps >= ctx->opts.max_sweeps)
        return fail(ctx, PCOL_E_SWEEPS, "sweep cap reached with pairs still resolving");
      // next sweep: new partners for DIRTY spheres (partner collided elsewhere)
      PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
      if (!ctx->small) {
        PCOL_HIP(launch_slot_min(s, n, 0, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                                 ctx->perm, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d));
        PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec,
                                     ctx->start, ctx->G, dt, ctx->status, ctx->perm, ctx->key_j,
                                     ctx->key_t));
      } else {
        PCOL_HIP(launch_gather_exact(s, nullptr, n, nullptr, ST_DIRTY, ctx->rec, ctx->start,
                                     ctx->G, dt, ctx->status, ctx->perm, ctx->key_j,
                                     ctx->key_t));
      }
    }
    if (timing) PCOL_HIP(hipEventRecord(ctx->ev[3], s));
    PCOL_HIP(launch_advance_sorted(s, n, ctx->rec, ctx->status, dt, ctx->G, ctx->out));
    PCOL_HIP(launch_unpermute(s, P, ctx->rank, ctx->out, part, tc));
    if (timing) {
      PCOL_HIP(hipEventRecord(ctx->ev[4], s));
      PCOL_HIP(hipEventSynchronize(ctx->ev[4]));
      ms_detect = ctx->detect_timed ? ms_between(ctx->ev[5], ctx->ev[6])
                                    : ms_between(ctx->ev[1], ctx->ev[2]);
    }
  }
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_pairs = pairs;
    stats->n_sweeps = sweeps;
    stats->contacts = (int64_t)contacts;
    stats->n_overflow = ovf_total;
    stats->n_recheck = (int64_t)recheck;
    stats->band = ctx->band;
    for (int a = 0; a < 3; ++a) {
      stats->nc[a] = ctx->G.nc[a];
      stats->h[a] = ctx->h[a];
    }
    stats->max_cell = ctx->maxcell;
    stats->home_cells = 1;
    stats->reach = ctx->reach;
    if (n > 0 && !ctx->small) {
      PCOL_HIP(hipMemsetAsync(ctx->tests_d, 0, sizeof(unsigned long long), s));
      PCOL_HIP(launch_count_pairs(s, ctx->start, ctx->G, ctx->tests_d));
      PCOL_HIP(hipMemcpyAsync(ctx->tests_h, ctx->tests_d, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
      PCOL_HIP(hipStreamSynchronize(s));
      stats->pair_tests = (int64_t)*ctx->tests_h;
    }
    if (timing && n > 0) {
      stats->ms_bin = ms_between(ctx->ev[0], ctx->ev[1]);
      stats->ms_detect = ms_detect;
      stats->ms_sweeps = ms_between(ctx->ev[2], ctx->ev[3]);
      stats->ms_advance = ms_between(ctx->ev[3], ctx->ev[4]);
    }
  }
  return PCOL_OK;
}

pcol_status pcol_step_backward(pcol_ctx *ctx, const pcol_particles *start, const pcol_box *box,
                               double dt, double e, const int32_t *partner, const double *tcoll,
                               const pcol_state_grad *g_out, pcol_state_grad *g_in, double *ge) {
  pcol_status st = check_common(ctx, start, box, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  if (!g_out || !g_in || !ge) return fail(ctx, PCOL_E_INVALID, "null gradient argument");
  if (start->n > 0 && (!partner || !tcoll || !g_out->x || !g_out->y || !g_out->z || !g_out->vx ||
                       !g_out->vy || !g_out->vz || !g_in->x || !g_in->y || !g_in->z ||
                       !g_in->vx || !g_in->vy || !g_in->vz))
    return fail(ctx, PCOL_E_INVALID, "null array");
  Grid G{};
  for (int a = 0; a < 3; ++a) {
    G.L[a] = box->len[a];
    G.halfL[a] = 0.5 * box->len[a];
  }
  StateGrad go{g_out->x, g_out->y, g_out->z, g_out->vx, g_out->vy, g_out->vz};
  StateGrad gi{g_in->x, g_in->y, g_in->z, g_in->vx, g_in->vy, g_in->vz};
  PCOL_HIP(launch_step_backward(ctx->stream, to_dev(start), G, dt, e, partner, tcoll, go, gi,
                                ctx->key_t, ge));
  return PCOL_OK;
}

}  // extern "C"
