// C-ABI layer of the pcol library: argument checks, the context and its
// device scratch, the grid choice, and the sweep driver of pcol_step.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

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
  int *rank = nullptr;  // caller index -> sorted position
  int *cid = nullptr;
  int *slot = nullptr;
  int *count = nullptr;
  int *start = nullptr;
  int *blocksum = nullptr;
  int64_t cell_cap = 0;
  CellCount *cellc = nullptr;  // per-cell counts of the detect kernels
  int64_t cellc_cap = 0;

  // sweep state
  int *cnt = nullptr;
  double *slot_t = nullptr;
  int *slot_j = nullptr;
  int *key_j = nullptr;
  double *key_t = nullptr;
  uint8_t *status = nullptr;
  int *ovf = nullptr;
  int *list_a = nullptr;  // spheres still to act after sweep 1
  int *keep_cnt = nullptr, *keep_off = nullptr, *keep_bs = nullptr;  // its construction
  int *nlist_h = nullptr;  // pinned read-back of its length
  OutRec *out = nullptr;
  int *partner_tmp = nullptr;
  double *tcoll_tmp = nullptr;
  ReachOut *reach_d = nullptr;
  ReachPart *reach_parts = nullptr;     // REACH_BLOCKS partial results of the reach pass
  unsigned int *reach_phist = nullptr;  // REACH_BLOCKS partial extent histograms
  SweepCounters *ctr_d = nullptr;
  ReachOut *reach_h = nullptr;
  SweepCounters *ctr_h = nullptr;
  // sweeps 2 on run on the device in groups: FLAG_* words and totals (pairs,
  // contacts, overflow) with their pinned read-back
  unsigned int *sflags = nullptr, *sflags_h = nullptr;
  unsigned long long *stotals = nullptr, *stotals_h = nullptr;
  hipEvent_t ev[8] = {};

  bool binned = false;
  int64_t binned_n = -1;
  const double *binned_x = nullptr;
  Grid G{};
  double reach = 0.0;
  double vmax = 0.0, rmin = 0.0, rmax = 0.0;
  double binned_dt = 0.0;
  // extent split: spheres with r + |v| dt > rho_c live in a second layer of
  // cells; the first layer's pair test then needs cells of side 2 rho_c only
  bool split = false;
  double rho_c = INFINITY, rho_max = 0.0;
  int wide_first = 0, n_wide = 0;  // sorted range of the second layer
  int *wide_h = nullptr;           // pinned read-back of that range
  bool bin_pending = false;        // maxcell and the range still in flight (bin_readback)
  const Spin *spin = nullptr;      // set by pcol_step_spin for the step: its spins are validated
  int walls = 0;                   // set by pcol_step_walls for the step: bit k = walls on axis k
  // pcol_deposit: position check flag, and the element sort's scratch with its capacities
  unsigned int *dep_flag_h = nullptr;
  unsigned char *dep_buf = nullptr;  // carved by deposit_layout
  int64_t dep_cap = 0;
  // bounds for the first layer's pair test: reach, speed and radius
  double reach_pass = 0.0, vmax_pass = 0.0, rmax_pass = 0.0;
  double band = 0.0;   // FP32 filter band in use (relative to r_i + r_j)
  double h[3] = {0, 0, 0};
  int maxcell = 0;
  bool small = false;  // some axis has fewer than 3 cells
  // the last binning's grid, tried first by the next call of the same shape
  // (sphere count, box, step, walls): its reach pass then bins on it as well
  bool plan_valid = false;
  int64_t plan_n = -1;
  double plan_L[3] = {0, 0, 0}, plan_dt = 0.0;
  int plan_walls = 0;
  Grid plan_G{};
  double plan_rho_c = INFINITY;
  bool detect_timed = false;
  int cpw_used = 0;  // home cells per workgroup of the last sweep-1 detect (0: exact search)
  unsigned long long *crank = nullptr;  // literal order (opts.order = 1): curve rank per sorted sphere
  struct BatchPlan *bp = nullptr;  // batched form (pcol_step_batched)
};

// State of the batched form: per-box grids on the host and device, the
// captured step graph and what it was captured for.
struct BatchPlan {
  // layout the tables were built for
  int nbox = 0;
  int64_t n = 0;
  std::vector<int64_t> box_off;
  std::vector<double> len;  // 3 per box
  // device tables
  Grid *gtab = nullptr;
  int *cell_base = nullptr;
  int *box_of = nullptr;
  int64_t *box_off_d = nullptr;
  double *breach = nullptr;
  int *chunk_box = nullptr;               // chunks of the reach pass (BREACH_CHUNK spheres)
  int64_t *chunk_lo = nullptr;
  BoxMax *bmax = nullptr;                 // [nbox], zero between passes
  int nchunk = 0, cap_chunk = 0;
  std::vector<int> chunk_box_h;
  std::vector<int64_t> chunk_lo_h;
  unsigned int *flags = nullptr;          // FLAG_* words
  unsigned long long *totals = nullptr;   // pairs, contacts, overflow
  int cap_box = 0;
  int64_t cap_n = 0;
  unsigned int *flags_h = nullptr;        // pinned: 4 flags + padding, then 3 totals
  std::vector<double> breach_h;
  std::vector<Grid> gtab_h;
  std::vector<int> cell_base_h;
  int total_cells = 0;
  bool tables = false;  // grids planned for the current layout
  // tuning choice
  double cell_mult = 1.0;
  int cpw = 4;           // home cells per workgroup of the pair-test launch
  bool tuned = false;
  int kmax = 12;        // sweeps captured in the graph
  // captured graph and its arguments
  hipStream_t gstream = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;
  const void *cap_ptr[8] = {};
  const void *cap_part = nullptr, *cap_tc = nullptr;
  double cap_dt = 0.0, cap_e = 0.0;
  // tuning scratch
  double *tune_buf = nullptr;
  int64_t tune_cap = 0;
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

// (re)allocate *p for at least `want` elements when its capacity `cap` is short
template <typename T>
hipError_t grow(T **p, int64_t &cap, int64_t want) {
  if (*p && cap >= want) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  cap = 0;
  const hipError_t e = hipMalloc((void **)p, (size_t)(want > 0 ? want : 1) * sizeof(T));
  if (e == hipSuccess) cap = want;
  return e;
}

double ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

// ---------------------------------------------------------------- deposition scratch

// The deposition's scratch carved out of one buffer, each part on a 256-B
// boundary: element id and slot per sphere, the element-sorted records, the
// per-element counts, starts and scan block sums, the scan's statistics word and
// the position flag.
struct DepositLayout {
  int64_t eid, slot, rec, cnt, start, bsum, ro, flag, bytes;
};

DepositLayout deposit_layout(int64_t n, int64_t ne, int comp) {
  DepositLayout L{};
  int64_t at = 0;
  auto take = [&at](int64_t bytes) {
    const int64_t here = at;
    at += (bytes + 255) / 256 * 256;
    return here;
  };
  L.eid = take(n * (int64_t)sizeof(int));
  L.slot = take(n * (int64_t)sizeof(int));
  L.rec = take(n * deposit_record_bytes(comp));
  L.cnt = take((ne + 1) * (int64_t)sizeof(int));
  L.start = take((ne + 1) * (int64_t)sizeof(int));
  L.bsum = take((ne / 4096 + 2) * (int64_t)sizeof(int));
  L.ro = take((int64_t)sizeof(ReachOut));
  L.flag = take((int64_t)sizeof(unsigned int));
  L.bytes = at;
  return L;
}

// Argument checks of the deposition (no device access); fills D but its
// scratch pointers.
pcol_status deposit_args(const double *x, const double *y, const double *z, int64_t n,
                         const double *a, int comp, const int32_t nc[3], const double len[3],
                         double *out, DepositArgs &D, const char *&why) {
  if (n < 0 || n > INT32_MAX) return why = "n outside [0, 2^31 - 1]", PCOL_E_INVALID;
  if (comp < 1 || comp > 8) return why = "comp outside [1, 8]", PCOL_E_INVALID;
  if (!nc || !len || !out) return why = "null grid or output", PCOL_E_INVALID;
  if (n > 0 && (!x || !y || !z || !a)) return why = "null array", PCOL_E_INVALID;
  D.x = x;
  D.y = y;
  D.z = z;
  D.a = a;
  D.n = n;
  D.comp = comp;
  D.out = out;
  D.nnode = 1;
  for (int d = 0; d < 3; ++d) {
    if (nc[d] < 1 || nc[d] > (1 << 20)) return why = "nc outside [1, 2^20]", PCOL_E_INVALID;
    if (!(len[d] > 0.0) || !isfinite(len[d])) return why = "box side <= 0", PCOL_E_INVALID;
    D.nc[d] = nc[d];
    D.L[d] = len[d];
    D.h[d] = len[d] / nc[d];
    D.nnode *= nc[d];
    if (D.nnode > INT32_MAX) return why = "more than 2^31 - 1 elements", PCOL_E_INVALID;
  }
  return PCOL_OK;
}

// The deposition on stream s with its scratch at base (laid out by Lo): the
// count checks every position and is read back (into flag_h, host memory)
// before anything of the caller's is written; st receives PCOL_E_INVALID for a
// bad position, else PCOL_OK.  Counts and the flag are cleared by fill kernels.
hipError_t deposit_run(DepositArgs &D, const DepositLayout &Lo, unsigned char *base, hipStream_t s,
                       unsigned int *flag_h, pcol_status &st) {
  st = PCOL_OK;
  D.eid = (int *)(base + Lo.eid);
  D.slot = (int *)(base + Lo.slot);
  D.rec = base + Lo.rec;
  D.cnt = (int *)(base + Lo.cnt);
  D.start = (int *)(base + Lo.start);
  unsigned int *flag = (unsigned int *)(base + Lo.flag);
  hipError_t e = launch_fill_i32(s, D.cnt, 0, D.nnode);
  if (e != hipSuccess) return e;
  if (D.n > 0) {  // the count checks the positions; nothing of the caller's is written yet
    if ((e = launch_fill_u32(s, flag, 0u, 1)) != hipSuccess) return e;
    if ((e = launch_deposit_count(s, D, flag)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(flag_h, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (*flag_h) {
      st = PCOL_E_INVALID;
      return hipSuccess;
    }
  }
  if ((e = launch_scan(s, D.cnt, (int)D.nnode, D.start, (int *)(base + Lo.bsum),
                       (ReachOut *)(base + Lo.ro))) != hipSuccess)
    return e;
  return launch_deposit(s, D);
}

}  // namespace

// ---------------------------------------------------------------- static scratch

// Device scratch of pcol_deposit_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (its host
// name is a stand-in, not a device address): the device address of each GPU's
// copy comes from hipGetSymbolAddress, taken once per device on the first call
// with that device current.
static __device__ __align__(256) unsigned char scratch[PCOL_NOALLOC_SCRATCH_BYTES];

static constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static unsigned char *scratch_ptr[MAX_DEVICES] = {};

static hipError_t static_scratch(unsigned char **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = (unsigned char *)p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}


extern "C" {

void pcol_default_opts(pcol_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->cell_mult = 1.0;
  o->max_sweeps = 0;
  o->home_cells = 0;
  o->contact_slots = 12;
  o->filter = 0;
  o->band_rel = 1e-4;
  o->timing = 0;
  o->autotune = 1;
  o->split_quantile = 0.999;
  o->order = 0;
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
  void *dev[] = {ctx->rec,    ctx->rank,   ctx->cid,         ctx->slot,
                 ctx->count,  ctx->start,  ctx->blocksum, ctx->cnt,      ctx->slot_t,
                 ctx->slot_j, ctx->key_j,  ctx->key_t,  ctx->status,      ctx->out,
                 ctx->ovf,    ctx->partner_tmp, ctx->tcoll_tmp, ctx->list_a, ctx->keep_cnt, ctx->keep_off, ctx->keep_bs,
                 ctx->reach_d, ctx->cellc, ctx->ctr_d, ctx->sflags, ctx->stotals, ctx->dep_buf,
                 ctx->crank, ctx->reach_parts, ctx->reach_phist};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  if (ctx->reach_h) (void)hipHostFree(ctx->reach_h);
  if (ctx->ctr_h) (void)hipHostFree(ctx->ctr_h);
  if (ctx->wide_h) (void)hipHostFree(ctx->wide_h);
  if (ctx->sflags_h) (void)hipHostFree(ctx->sflags_h);
  if (ctx->stotals_h) (void)hipHostFree(ctx->stotals_h);
  if (ctx->nlist_h) (void)hipHostFree(ctx->nlist_h);
  if (ctx->dep_flag_h) (void)hipHostFree(ctx->dep_flag_h);
  for (hipEvent_t &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (BatchPlan *bp = ctx->bp) {
    void *bd[] = {bp->gtab,    bp->cell_base, bp->box_of, bp->box_off_d, bp->breach,
                  bp->chunk_box, bp->chunk_lo, bp->bmax,  bp->flags,     bp->totals,
                  bp->tune_buf};
    for (void *q : bd)
      if (q) (void)hipFree(q);
    if (bp->flags_h) (void)hipHostFree(bp->flags_h);
    if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
    if (bp->gstream) (void)hipStreamDestroy(bp->gstream);
    delete bp;
  }
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
      ctx->opts.home_cells < 0 || ctx->opts.home_cells > 16 ||
      ctx->opts.order < 0 || ctx->opts.order > 1 ||
      !(ctx->opts.band_rel >= 0.0) ||
      !(ctx->opts.split_quantile >= 0.0 && ctx->opts.split_quantile <= 1.0) ||
      ctx->opts.filter < 0 || ctx->opts.filter > 1) {
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
  A(dalloc(&ctx->list_a, n));
  A(dalloc(&ctx->keep_cnt, n / 256 + 2));
  A(dalloc(&ctx->keep_off, n / 256 + 3));
  A(dalloc(&ctx->keep_bs, n / 256 / 4096 + 2));
  A(dalloc(&ctx->partner_tmp, n));
  A(dalloc(&ctx->tcoll_tmp, n));
  if (ctx->opts.order == 1) A(dalloc(&ctx->crank, n));
  A(dalloc(&ctx->reach_d, 1));
  A(dalloc(&ctx->reach_parts, REACH_BLOCKS));
  A(dalloc(&ctx->reach_phist, (int64_t)REACH_BLOCKS * RHO_BINS));
  A(dalloc(&ctx->ctr_d, 1));
  A(dalloc(&ctx->sflags, 16));
  A(dalloc(&ctx->stotals, 4));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->sflags_h, 16 * sizeof(unsigned int));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->stotals_h, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->reach_h, sizeof(ReachOut));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->ctr_h, sizeof(SweepCounters));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->wide_h, 2 * sizeof(int));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->nlist_h, sizeof(int));
  for (hipEvent_t &ev : ctx->ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    pcol_destroy(ctx);
    return e == hipErrorOutOfMemory ? PCOL_E_NOMEM : PCOL_E_HIP;
  }
  *out = ctx;
  return PCOL_OK;
}

// Host copies of the largest cell occupancy and the second layer's range,
// once the read-backs pcol_bin queued have landed (after a stream
// synchronisation).
static void bin_readback(pcol_ctx *ctx) {
  if (!ctx->bin_pending) return;
  ctx->maxcell = (int)ctx->reach_h->maxcell;
  ctx->wide_first = ctx->split ? ctx->wide_h[0] : (int)ctx->binned_n;
  ctx->n_wide = (int)ctx->binned_n - ctx->wide_first;
  ctx->bin_pending = false;
}

pcol_status pcol_bin(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box, double dt) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  ctx->binned = false;
  Particles P = to_dev(p);
  if (ctx->spin) {
    P.wx = ctx->spin->wx;
    P.wy = ctx->spin->wy;
    P.wz = ctx->spin->wz;
  }
  hipStream_t s = ctx->stream;
  // The grid of the last binning is tried first when this call has its shape
  // (sphere count, box, step, walls): the reach pass then also takes every
  // sphere's cell and slot on it (a2), and the plan is kept only if the reach
  // now measured leads to the same grid and split extent; otherwise the counts
  // are redone on the new grid below.  Either way the grid is the one the
  // reach of this call determines.
  const bool tried = ctx->plan_valid && ctx->plan_n == p->n && ctx->plan_dt == dt &&
                     ctx->plan_walls == ctx->walls && ctx->plan_L[0] == box->len[0] &&
                     ctx->plan_L[1] == box->len[1] && ctx->plan_L[2] == box->len[2] &&
                     (int64_t)(ctx->plan_G.layer2 ? 2 * ctx->plan_G.ncell : ctx->plan_G.ncell) +
                             2 <= ctx->cell_cap;
  ctx->plan_valid = false;
  // a1: reach and data validity (one read-back); the histogram is accumulated
  // into zeros, the other fields are written by the reduction
  PCOL_HIP(hipMemsetAsync(ctx->reach_d, 0, sizeof(ReachOut), s));
  // the extent histogram only picks the split extent: above 2^20 spheres it
  // samples one sphere in 16 (the quantile of a million samples is as good)
  const int hist_shift = p->n >= (1 << 20) ? 4 : 0;
  if (tried) {
    const Grid &T = ctx->plan_G;
    PCOL_HIP(launch_fill_i32(s, ctx->count, 0, T.layer2 ? 2 * T.ncell : T.ncell));
    PCOL_HIP(launch_reach(s, P, box->len, dt, hist_shift, ctx->reach_d, ctx->reach_parts,
                          ctx->reach_phist, &T, ctx->plan_rho_c, ctx->cid, ctx->slot,
                          ctx->count));
  } else {
    PCOL_HIP(launch_reach(s, P, box->len, dt, hist_shift, ctx->reach_d, ctx->reach_parts,
                          ctx->reach_phist));
  }
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
  double rho_max;
  memcpy(&rho_max, &ro.rhomax, sizeof(double));
  // Extent split: the first layer holds the spheres whose extent is at most
  // rho_c, the upper edge of the histogram bin where the split quantile of the
  // extents falls; pairs of them are at most 2 rho_c apart when they can touch.
  // Used only when it shrinks the cells enough to pay for the separate search
  // of the others, and the grid keeps 3 cells per axis.
  double rho_c = INFINITY;
  const double q = ctx->opts.split_quantile;
  double sampled = 0.0;
  for (int k = 0; k < RHO_BINS; ++k) sampled += ro.hist[k];
  if (q > 0.0 && q < 1.0 && p->n >= 4096) {
    const double target = ceil(q * sampled);
    double cum = 0.0;
    for (int k = 0; k < RHO_BINS - 1; ++k) {
      cum += ro.hist[k];
      if (cum >= target) {
        // upper edge of bin k: the lower edge of bin k + 1
        const uint64_t top = (uint64_t)((1023 - 64) * 16 + k + 1);
        const uint64_t bits = top << 48;
        memcpy(&rho_c, &bits, sizeof(double));
        break;
      }
    }
    if (!(2.0 * rho_c < 0.85 * reach)) rho_c = INFINITY;
    for (int a = 0; a < 3 && isfinite(rho_c); ++a)
      if (box->len[a] / (2.0 * rho_c * ctx->opts.cell_mult * (1.0 + 1e-9)) < 3.0) rho_c = INFINITY;
  }
  const bool split = isfinite(rho_c);
  const double reach_pass = split ? 2.0 * rho_c : reach;
  // grid: cell side >= (split ? 2 rho_c : reach) * cell_mult, at most 2^26 cells per layer
  Grid G{};
  double cell = reach_pass * ctx->opts.cell_mult;
  if (!(cell > 0.0)) cell = box->len[0];  // no motion and no size: one cell
  for (;;) {
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
      double q3 = floor(box->len[a] / (cell * (1.0 + 1e-9)));
      if (!(q3 >= 1.0)) q3 = 1.0;
      if (q3 > 1024.0) q3 = 1024.0;
      G.nc[a] = (int)q3;
      ncell *= G.nc[a];
    }
    if (ncell <= (1 << 26)) {
      G.ncell = (int)ncell;
      break;
    }
    cell *= 1.25;
  }
  ctx->small = false;
  G.walls = ctx->walls;
  for (int a = 0; a < 3; ++a) {
    const bool wall = (ctx->walls >> a) & 1;
    G.L[a] = box->len[a];
    // between walls there is no minimum image and no periodic image shift
    G.halfL[a] = wall ? INFINITY : 0.5 * box->len[a];
    G.sL[a] = wall ? 0.0 : box->len[a];
    G.inv_h[a] = (double)G.nc[a] / box->len[a];
    G.h[a] = box->len[a] / G.nc[a];
    ctx->h[a] = G.h[a];
    if (G.nc[a] < 3) ctx->small = true;
  }
  G.layer2 = split ? G.ncell : 0;
  G.rho_max = split ? rho_max : 0.0;
  G.inv_row = 1.0 / G.nc[0];
  G.inv_layer = 1.0 / ((double)G.nc[0] * G.nc[1]);
  const int cells_all = split ? 2 * G.ncell : G.ncell;
  if ((int64_t)cells_all + 2 > ctx->cell_cap) {
    if (ctx->count) (void)hipFree(ctx->count);
    if (ctx->start) (void)hipFree(ctx->start);
    if (ctx->blocksum) (void)hipFree(ctx->blocksum);
    ctx->count = ctx->start = ctx->blocksum = nullptr;
    ctx->cell_cap = 0;
    if (ctx->bp) ctx->bp->captured = false;  // its graph holds the old cell arrays
    const int64_t cap = (int64_t)cells_all + 2;
    hipError_t e = dalloc(&ctx->count, (size_t)cap);
    if (e == hipSuccess) e = dalloc(&ctx->start, (size_t)cap + 1);
    if (e == hipSuccess) e = dalloc(&ctx->blocksum, (size_t)(cap / 4096 + 2));
    if (e != hipSuccess) return fail(ctx, PCOL_E_NOMEM, "cell arrays");
    ctx->cell_cap = cap;
  }
  // a2-a4: counting sort into cell-sorted records (the counts already taken by
  // the reach pass when the tried grid is this one)
  const bool binned_on_plan = tried && ctx->plan_G.nc[0] == G.nc[0] &&
                              ctx->plan_G.nc[1] == G.nc[1] && ctx->plan_G.nc[2] == G.nc[2] &&
                              ctx->plan_G.layer2 == G.layer2 &&
                              (!split || ctx->plan_rho_c == rho_c);
  if (!binned_on_plan) {
    PCOL_HIP(launch_fill_i32(s, ctx->count, 0, cells_all));
    PCOL_HIP(launch_cell_hist(s, P, G, dt, rho_c, ctx->cid, ctx->slot, ctx->count));
  }
  PCOL_HIP(launch_scan(s, ctx->count, cells_all, ctx->start, ctx->blocksum, ctx->reach_d));
  PCOL_HIP(launch_scatter(s, P, ctx->cid, ctx->slot, ctx->start, ctx->rec, ctx->rank, nullptr));
  if (ctx->opts.order == 1) {
    // the literal order's ranks on the curve grid: cell side >= the reach
    // (2 max r + 2 max|v| dt, whatever grid the pair tests use), at most 2048
    // cells per axis
    CurveGrid C{};
    for (int a = 0; a < 3; ++a) {
      double q3 = floor(box->len[a] / (reach * (1.0 + 1e-9)));
      if (!(q3 >= 1.0)) q3 = 1.0;
      if (q3 > 2048.0) q3 = 2048.0;
      C.nc[a] = (int)q3;
      C.h[a] = box->len[a] / C.nc[a];
    }
    PCOL_HIP(launch_curve_rank(s, ctx->rec, (int)p->n, C, ctx->crank));
  }
  // the largest cell and the second layer's range are read back without a
  // wait; they are read after the next synchronisation (bin_readback)
  PCOL_HIP(hipMemcpyAsync(&ctx->reach_h->maxcell, &ctx->reach_d->maxcell, sizeof(unsigned int),
                          hipMemcpyDeviceToHost, s));
  if (split)
    PCOL_HIP(hipMemcpyAsync(ctx->wide_h, ctx->start + G.layer2, sizeof(int), hipMemcpyDeviceToHost, s));
  ctx->bin_pending = true;
  ctx->G = G;
  ctx->reach = reach;
  ctx->vmax = sqrt(v2);
  ctx->rmin = rmin;
  ctx->rmax = rmax;
  ctx->binned_dt = dt;
  ctx->split = split;
  ctx->rho_c = rho_c;
  ctx->rho_max = rho_max;
  // first-layer bounds: extent <= rho_c gives |v| <= (rho_c - r_min) / dt, r <= rho_c
  ctx->reach_pass = reach_pass;
  ctx->vmax_pass = split ? std::min(ctx->vmax, (rho_c - rmin) / dt) : ctx->vmax;
  ctx->rmax_pass = split ? std::min(rmax, rho_c) : rmax;
  ctx->binned = true;
  ctx->binned_n = p->n;
  ctx->binned_x = p->x;
  ctx->plan_valid = true;
  ctx->plan_n = p->n;
  ctx->plan_dt = dt;
  ctx->plan_walls = ctx->walls;
  for (int a = 0; a < 3; ++a) ctx->plan_L[a] = box->len[a];
  ctx->plan_G = G;
  ctx->plan_rho_c = rho_c;
  return PCOL_OK;
}

static pcol_status check_binned(pcol_ctx *ctx, const pcol_particles *p, const pcol_box *box,
                                double dt) {
  if (!ctx->binned || ctx->binned_n != p->n)
    return fail(ctx, PCOL_E_STATE, "pcol_bin must run first on the same particle set");
  if (ctx->G.walls) return fail(ctx, PCOL_E_STATE, "the last binning was for a box with walls");
  if (dt != ctx->binned_dt) return fail(ctx, PCOL_E_STATE, "dt differs from pcol_bin");
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
  const double R = ctx->reach_pass, V = ctx->vmax_pass, smin = 2.0 * ctx->rmin;
  const double k0 = 1.0 + ctx->opts.band_rel + 1e-3;  // generous k for the radius term
  const double Dd = (2.0 * h + R) * u, Du = 4.0 * V * u;
  const double ec = 2.0 * sqrt(3.0) * R * Dd + 3.0 * u * R * R +
                    6.0 * u * (2.0 * ctx->rmax_pass * k0) * (2.0 * ctx->rmax_pass * k0);
  const double eb = (sqrt(3.0) * (R * Du + 2.0 * V * Dd) + 6.0 * u * R * V) * 2.0 * dt *
                    (1.0 + 0x1.0p-11);
  const double need = 2.0 * (ec + eb) / (2.0 * smin * smin);
  return ctx->opts.band_rel > need ? ctx->opts.band_rel : need;
}

// Tolerance of the binary64 Gram filter (filter 0).  The filter evaluates
// G = alpha_i + <P_j, Q_i> (seven FMAs from alpha_i) from coordinates relative
// to the home cell centre and passes the pair when G <= fl(tol - beta_j); in
// real numbers that is F = G + beta_j <= tol.  For a pair the rule keeps, the
// real F is at most E0 = 3 eps ((reach^2 + (2 r_max)^2) + reach 2 v_max dt2)
// (the binary64 argument: the kept root c / (-b + sqrt D) <= dt gives
// c <= 2 |b| dt (1 + 6 eps) < |b| dt2).  The evaluation differs from the real F by
//  * the relative coordinates: each is one or two roundings of values below
//    L + h, so the separation d is off by at most delta = eps (2 (Lmax + h) + X_i +
//    X_j), which moves F by at most delta (2 reach + 2 v_max dt2) + delta^2;
//  * alpha, beta, Q, P (a few roundings each, <= 6 eps relative) and the seven
//    FMAs of the sum (<= 7 eps of the sum of magnitudes): at most
//    16 eps (A_ + B_ + S) with A_, B_, S the bounds of |alpha|, |beta| and
//    sum_k |P_k Q_k| for |x_i| <= X_i = (sqrt 3 / 2) h, |x_j| <= X_i + reach;
//  * the threshold's one rounding, at most eps (tol + |beta|): the eps tol part
//    is covered by the factor two below, the eps B_ part by a 17th eps.
// The tolerance is twice the sum.
static double gram64_tolerance(double h, double R, double V, double r, double Lmax,
                               double dt2) {
  const double s3 = sqrt(3.0), eps = 0x1.0p-53;
  const double Xi = 0.5 * s3 * h * (1.0 + 1e-6), Xj = Xi + R;
  const double Ab = Xi * Xi + dt2 * Xi * V + r * r, Bb = Xj * Xj + dt2 * Xj * V + r * r;
  const double S = Xj * (2.0 * Xi + dt2 * V) + V * dt2 * Xi + 2.0 * r * r;
  const double E0 = 3.0 * eps * ((R * R + 4.0 * r * r) + R * 2.0 * V * dt2);
  const double delta = eps * (2.0 * (Lmax + h) + Xi + Xj);
  const double Epos = delta * (2.0 * R + 2.0 * V * dt2) + delta * delta;
  const double E = 17.0 * eps * (Ab + Bb + S);
  return 2.0 * (E0 + Epos + E);
}

// sweep 1: keys of all spheres (all active) into ctx->key_j / key_t (sorted
// order); crank given: the literal order's partners instead of rule 2's
static pcol_status detect_all(pcol_ctx *ctx, double dt, const unsigned long long *crank) {
  hipStream_t s = ctx->stream;
  const int n = (int)ctx->binned_n;
  if (!ctx->small) {
    if (ctx->G.ncell > ctx->cellc_cap) {
      if (ctx->cellc) (void)hipFree(ctx->cellc);
      ctx->cellc = nullptr;
      ctx->cellc_cap = 0;
      if (dalloc(&ctx->cellc, (size_t)ctx->G.ncell) != hipSuccess)
        return fail(ctx, PCOL_E_NOMEM, "cell counts");
      ctx->cellc_cap = ctx->G.ncell;
    }
    DetectArgs A{};
    A.cellc = ctx->cellc;
    // sparse cells (the split grid holds about 13 spheres per cell at 16M): four
    // cells per workgroup, so their survivors are decided together; opts.home_cells
    // overrides the choice
    A.cpw = ctx->opts.home_cells > 0 ? ctx->opts.home_cells
                                     : (n < 24 * (int64_t)ctx->G.ncell ? 4 : 1);
    ctx->cpw_used = A.cpw;
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
      const double R = ctx->reach_pass, smax = 2.0 * ctx->rmax_pass;
      A.tol = 16.0 * 0x1.0p-53 * (R * R + smax * smax + R * 2.0 * ctx->vmax_pass * A.dt2);
      double h = ctx->h[0], Lmax = ctx->G.L[0];
      for (int a = 1; a < 3; ++a) {
        h = ctx->h[a] > h ? ctx->h[a] : h;
        Lmax = ctx->G.L[a] > Lmax ? ctx->G.L[a] : Lmax;
      }
      A.tol64 = gram64_tolerance(h, R, ctx->vmax_pass, ctx->rmax_pass, Lmax, A.dt2);
      // pairs with a sphere above the split extent: |d| up to the full reach
      const double Rw = ctx->reach, sw = 2.0 * ctx->rmax;
      A.tol_wide = 16.0 * 0x1.0p-53 * (Rw * Rw + sw * sw + Rw * 2.0 * ctx->vmax * A.dt2);
      A.rho_c = ctx->rho_c;
    }
    A.K = ctx->K;
    A.fp32 = ctx->opts.filter == 1;
    ctx->band = A.fp32 ? fp32_band(ctx, dt) : 0.0;
    // round the factor up so the float never shrinks the inflation
    const double kb = 1.0 + ctx->band;
    A.kband = (float)kb;
    if ((double)A.kband < kb) A.kband = nextafterf(A.kband, 2.0f);
    A.dt2f = (float)(2.0 * dt * (1.0 + 0x1.0p-12));
    PCOL_HIP(launch_fill_i32(s, ctx->cnt, 0, n));
    if (ctx->opts.timing) PCOL_HIP(hipEventRecord(ctx->ev[5], s));
    PCOL_HIP(launch_detect_half(s, A));
    PCOL_HIP(launch_cell_counts(s, ctx->cellc, detect_half_blocks(A), ctx->ctr_d));
    // spheres of large extent: exact search of their wider neighbourhood
    if (ctx->split) PCOL_HIP(launch_detect_wide(s, A, ctx->start + ctx->G.layer2, n));
    if (ctx->opts.timing) PCOL_HIP(hipEventRecord(ctx->ev[6], s));
    ctx->detect_timed = true;
    PCOL_HIP(launch_slot_min(s, n, 1, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                             ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d,
                             nullptr, nullptr, 0, &ctx->G, crank));
    PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec, ctx->start,
                                 ctx->G, dt, ctx->status, ctx->key_j, ctx->key_t, nullptr, crank));
  } else {
    // fewer than 3 cells on some axis: exact search for every sphere
    ctx->cpw_used = 0;
    PCOL_HIP(launch_gather_exact(s, nullptr, n, nullptr, -1, ctx->rec, ctx->start, ctx->G, dt,
                                 ctx->status, ctx->key_j, ctx->key_t, nullptr, crank));
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
  if ((st = check_binned(ctx, p, box, dt)) != PCOL_OK) return st;
  if (p->n > 0 && !key_out) return fail(ctx, PCOL_E_INVALID, "key_out is null");
  hipStream_t s = ctx->stream;
  const int n = (int)p->n;
  if (n == 0) return PCOL_OK;
  PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
  if (!active) {
    PCOL_HIP(launch_fill_u8(s, ctx->status, ST_ACTIVE, n));
    if ((st = detect_all(ctx, dt, nullptr)) != PCOL_OK) return st;
  } else {
    PCOL_HIP(launch_status_from_active(s, active, ctx->rec, n, ctx->status));
    PCOL_HIP(launch_fill_i32(s, ctx->key_j, -1, n));
    PCOL_HIP(launch_gather_exact(s, nullptr, n, nullptr, ST_ACTIVE, ctx->rec, ctx->start, ctx->G,
                                 dt, ctx->status, ctx->key_j, ctx->key_t, nullptr));
  }
  PCOL_HIP(launch_export_keys(s, n, ctx->rec, ctx->key_j, ctx->key_t, ctx->status, key_out,
                              tmin_out));
  return PCOL_OK;
}

pcol_status pcol_resolve(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                         double e, const uint64_t *key, uint8_t *active, int32_t *partner,
                         double *tcoll, int64_t *n_pairs_dev) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  if ((st = check_binned(ctx, p, box, dt)) != PCOL_OK) return st;
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

}  // extern "C"

// The whole step of pcol_step and pcol_step_spin (spin: nullptr for none).
static pcol_status step_impl(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt,
                             double e, int32_t *partner, double *tcoll, pcol_stats *stats,
                             const Spin *spin) {
  pcol_status st = check_common(ctx, p, box, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  if (ctx->opts.order == 1 && (spin || ctx->walls))
    return fail(ctx, PCOL_E_INVALID, "the literal order (opts.order = 1) is built for pcol_step only");
  // the literal order's ranks (set by the binning), else rule 2
  const unsigned long long *crank = ctx->opts.order == 1 ? ctx->crank : nullptr;
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
  unsigned long long contacts = 0ull, recheck = 0ull, tests = 0ull;
  double ms_detect = 0.0;
  if (n > 0) {
    PCOL_HIP(launch_fill_u8(s, ctx->status, ST_ACTIVE, n));
    PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
    // sweep 1: every contact within dt, then the earliest partner of each sphere
    ctx->detect_timed = false;
    if ((st = detect_all(ctx, dt, crank)) != PCOL_OK) return st;
    if (timing) PCOL_HIP(hipEventRecord(ctx->ev[2], s));
    // sweep 1 over every sphere; later sweeps over the list of the spheres it
    // left ACTIVE or DIRTY (the others are done for the step; entries that
    // finish later are skipped by their status)
    PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, P.m, ctx->key_j, ctx->key_t,
                                  ctx->status, ctx->out, ctx->ctr_d, nullptr,
                                  nullptr, 0, spin));
    PCOL_HIP(launch_keep_list(s, ctx->status, n, ctx->keep_cnt, ctx->keep_off, ctx->keep_bs,
                              ctx->reach_d, ctx->list_a));
    PCOL_HIP(hipMemcpyAsync(ctx->nlist_h, ctx->keep_off + (n + 255) / 256, sizeof(int),
                            hipMemcpyDeviceToHost, s));
    PCOL_HIP(hipMemcpyAsync(ctx->ctr_h, ctx->ctr_d, sizeof(SweepCounters), hipMemcpyDeviceToHost,
                            s));
    PCOL_HIP(hipStreamSynchronize(s));
    bin_readback(ctx);
    {
      unsigned long long sp, sc;
      sum_counters(*ctx->ctr_h, sp, sc);
      contacts = sc / 2ull;
      for (int k = 0; k < NSHARD; ++k) {
        recheck += ctx->ctr_h->shard[k].recheck;
        tests += ctx->ctr_h->shard[k].tests;
      }
      ovf_total = ctx->ctr_h->n_overflow;
      sweeps = 1;
      pairs = (int64_t)sp;
    }
    const int *lin = ctx->list_a;
    const int nlist = *ctx->nlist_h;
    // Later sweeps over a long list run on the device in groups without a host
    // round trip per sweep: each ends with k_sweep_check, which totals its pairs
    // and, at zero, raises FLAG_DONE, turning every later kernel into an early
    // exit.  The group's last check raises FLAG_UNFINISHED if that sweep still
    // paired, so the free flight queued behind the group only runs once the step
    // is done.  A short list (small boxes, where launches cost more than the
    // kernels) takes one sweep per round trip, with no launches to spare.
    BatchDev Bf{};
    Bf.flags = ctx->sflags;
    const bool more = pairs > 0;
    const bool groups = nlist >= (1 << 16);
    if (more && ctx->opts.max_sweeps == 1)
      return fail(ctx, PCOL_E_SWEEPS, "sweep cap reached with pairs still resolving");
    while (more && !groups) {
      PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
      if (!ctx->small) {
        PCOL_HIP(launch_slot_min(s, n, 0, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K,
                                 ctx->status, ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf,
                                 ctx->ctr_d, nullptr, lin, nlist, &ctx->G, crank));
        PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec,
                                     ctx->start, ctx->G, dt, ctx->status, ctx->key_j,
                                     ctx->key_t, nullptr, crank));
      } else {
        PCOL_HIP(launch_gather_exact(s, lin, nlist, nullptr, ST_DIRTY, ctx->rec, ctx->start,
                                     ctx->G, dt, ctx->status, ctx->key_j, ctx->key_t, nullptr,
                                     crank));
      }
      PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, P.m, ctx->key_j, ctx->key_t,
                                    ctx->status, ctx->out, ctx->ctr_d, nullptr,
                                    lin, nlist, spin));
      PCOL_HIP(hipMemcpyAsync(ctx->ctr_h, ctx->ctr_d, sizeof(SweepCounters),
                              hipMemcpyDeviceToHost, s));
      PCOL_HIP(hipStreamSynchronize(s));
      unsigned long long sp, sc;
      sum_counters(*ctx->ctr_h, sp, sc);
      ovf_total += ctx->ctr_h->n_overflow;
      ++sweeps;
      pairs += (int64_t)sp;
      if (sp == 0ull) break;
      if (ctx->opts.max_sweeps > 0 && sweeps >= ctx->opts.max_sweeps)
        return fail(ctx, PCOL_E_SWEEPS, "sweep cap reached with pairs still resolving");
    }
    if (more && groups) {
      PCOL_HIP(launch_fill_u32(s, ctx->sflags, 0u, 16));
      PCOL_HIP(launch_fill_u32(s, (unsigned int *)ctx->stotals, 0u, 8));
      PCOL_HIP(hipMemsetAsync(ctx->ctr_d, 0, sizeof(SweepCounters), s));
    }
    for (int group = 0; more && groups; ++group) {
      int S = group == 0 ? 5 : 2;  // a step takes about six sweeps at 16M
      if (ctx->opts.max_sweeps > 0 && S > ctx->opts.max_sweeps - (int)sweeps)
        S = ctx->opts.max_sweeps - (int)sweeps;
      for (int k = 0; k < S; ++k) {
        // new partners for DIRTY spheres (partner collided elsewhere), then the resolve
        if (!ctx->small) {
          PCOL_HIP(launch_slot_min(s, n, 0, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K,
                                   ctx->status, ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf,
                                   ctx->ctr_d, ctx->sflags, lin, nlist, &ctx->G, crank));
          PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec,
                                       ctx->start, ctx->G, dt, ctx->status, ctx->key_j,
                                       ctx->key_t, &Bf, crank));
        } else {
          PCOL_HIP(launch_gather_exact(s, lin, nlist, nullptr, ST_DIRTY, ctx->rec, ctx->start,
                                       ctx->G, dt, ctx->status, ctx->key_j, ctx->key_t, &Bf,
                                       crank));
        }
        PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, P.m, ctx->key_j,
                                      ctx->key_t, ctx->status, ctx->out, ctx->ctr_d, &Bf,
                                      lin, nlist, spin));
        PCOL_HIP(launch_sweep_check(s, ctx->ctr_d, ctx->sflags, ctx->stotals, k == S - 1));
      }
      if (timing) PCOL_HIP(hipEventRecord(ctx->ev[3], s));
      PCOL_HIP(launch_finish(s, P, ctx->rank, ctx->out, ctx->status, part, tc, dt, ctx->G,
                             &Bf));
      PCOL_HIP(hipMemcpyAsync(ctx->sflags_h, ctx->sflags, 4 * sizeof(unsigned int),
                              hipMemcpyDeviceToHost, s));
      PCOL_HIP(hipMemcpyAsync(ctx->stotals_h, ctx->stotals, 3 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
      PCOL_HIP(hipStreamSynchronize(s));
      if (ctx->sflags_h[FLAG_DONE]) break;
      if (ctx->opts.max_sweeps > 0 && 1 + (int)ctx->sflags_h[FLAG_SWEEPS] >= ctx->opts.max_sweeps)
        return fail(ctx, PCOL_E_SWEEPS, "sweep cap reached with pairs still resolving");
      sweeps = 1 + ctx->sflags_h[FLAG_SWEEPS];
      PCOL_HIP(launch_fill_u32(s, ctx->sflags + FLAG_UNFINISHED, 0u, 1));
    }
    if (more && groups) {
      sweeps = 1 + ctx->sflags_h[FLAG_SWEEPS];
      pairs += (int64_t)ctx->stotals_h[0];
      ovf_total += (int64_t)ctx->stotals_h[2];
    } else {
      if (timing) PCOL_HIP(hipEventRecord(ctx->ev[3], s));
      PCOL_HIP(launch_finish(s, P, ctx->rank, ctx->out, ctx->status, part, tc, dt, ctx->G,
                             nullptr));
    }
    if (timing) {
      PCOL_HIP(hipEventRecord(ctx->ev[4], s));
      PCOL_HIP(hipEventSynchronize(ctx->ev[4]));
      ms_detect = ctx->detect_timed ? ms_between(ctx->ev[5], ctx->ev[6])
                                    : ms_between(ctx->ev[1], ctx->ev[2]);
    }
  }
  if (stats) {
    if (ctx->bin_pending) {  // an empty step: nothing waited for the read-backs yet
      PCOL_HIP(hipStreamSynchronize(s));
      bin_readback(ctx);
    }
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
    stats->home_cells = ctx->cpw_used;
    stats->reach = ctx->reach;
    stats->n_wide = ctx->n_wide;
    stats->rho_c = ctx->split ? ctx->rho_c : 0.0;
    stats->pair_tests = (int64_t)tests;
    if (timing && n > 0) {
      stats->ms_bin = ms_between(ctx->ev[0], ctx->ev[1]);
      stats->ms_detect = ms_detect;
      stats->ms_sweeps = ms_between(ctx->ev[2], ctx->ev[3]);
      stats->ms_advance = ms_between(ctx->ev[3], ctx->ev[4]);
    }
  }
  return PCOL_OK;
}

extern "C" {

pcol_status pcol_step(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box, double dt, double e,
                      int32_t *partner, double *tcoll, pcol_stats *stats) {
  return step_impl(ctx, p, box, dt, e, partner, tcoll, stats, nullptr);
}

pcol_status pcol_step_spin(pcol_ctx *ctx, pcol_particles *p, double *wx, double *wy, double *wz,
                           const pcol_box *box, double dt, double e, double mu,
                           int32_t *partner, double *tcoll, pcol_stats *stats) {
  if (!ctx) return PCOL_E_INVALID;
  if (!(mu >= 0.0) || !isfinite(mu)) return fail(ctx, PCOL_E_INVALID, "mu negative or not finite");
  if (p && p->n > 0 && (!wx || !wy || !wz)) return fail(ctx, PCOL_E_INVALID, "null spin array");
  const Spin sp{wx, wy, wz, mu};
  ctx->spin = &sp;  // the binning validates the spins with the other inputs
  const pcol_status st = step_impl(ctx, p, box, dt, e, partner, tcoll, stats, &sp);
  ctx->spin = nullptr;
  return st;
}

pcol_status pcol_step_spin_walls(pcol_ctx *ctx, pcol_particles *p, double *wx, double *wy,
                                 double *wz, const pcol_box *box, const int32_t walls[3],
                                 double dt, double e, double mu, int32_t *partner, double *tcoll,
                                 pcol_stats *stats) {
  if (!ctx) return PCOL_E_INVALID;
  if (!walls) return fail(ctx, PCOL_E_INVALID, "null walls");
  int mask = 0;
  for (int a = 0; a < 3; ++a)
    if (walls[a]) mask |= 1 << a;
  ctx->walls = mask;
  const pcol_status st = pcol_step_spin(ctx, p, wx, wy, wz, box, dt, e, mu, partner, tcoll, stats);
  ctx->walls = 0;
  return st;
}

pcol_status pcol_step_walls(pcol_ctx *ctx, pcol_particles *p, const pcol_box *box,
                            const int32_t walls[3], double dt, double e, int32_t *partner,
                            double *tcoll, pcol_stats *stats) {
  if (!ctx) return PCOL_E_INVALID;
  if (!walls) return fail(ctx, PCOL_E_INVALID, "null walls");
  int mask = 0;
  for (int a = 0; a < 3; ++a)
    if (walls[a]) mask |= 1 << a;
  ctx->walls = mask;  // the binning builds its grid with these walls
  const pcol_status st = step_impl(ctx, p, box, dt, e, partner, tcoll, stats, nullptr);
  ctx->walls = 0;
  return st;
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
    G.sL[a] = box->len[a];
  }
  StateGrad go{g_out->x, g_out->y, g_out->z, g_out->vx, g_out->vy, g_out->vz};
  StateGrad gi{g_in->x, g_in->y, g_in->z, g_in->vx, g_in->vy, g_in->vz};
  PCOL_HIP(launch_step_backward(ctx->stream, to_dev(start), G, dt, e, partner, tcoll, go, gi,
                                ctx->key_t, ge));
  return PCOL_OK;
}

pcol_status pcol_deposit(pcol_ctx *ctx, const double *x, const double *y, const double *z,
                         int64_t n, const double *a, int comp, const int32_t nc[3],
                         const double len[3], double *out) {
  if (!ctx) return PCOL_E_INVALID;
  DepositArgs D{};
  const char *why = nullptr;
  pcol_status st = deposit_args(x, y, z, n, a, comp, nc, len, out, D, why);
  if (st != PCOL_OK) return fail(ctx, st, why);
  hipStream_t s = ctx->stream;
  const DepositLayout Lo = deposit_layout(D.n, D.nnode, comp);
  if (ctx->dep_cap < Lo.bytes || !ctx->dep_flag_h) {
    PCOL_HIP(hipStreamSynchronize(s));  // the free below waits for nothing queued
    hipError_t e = grow(&ctx->dep_buf, ctx->dep_cap, Lo.bytes);
    if (e == hipSuccess && !ctx->dep_flag_h)
      e = hipHostMalloc((void **)&ctx->dep_flag_h, sizeof(unsigned int));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, e == hipErrorOutOfMemory ? PCOL_E_NOMEM : PCOL_E_HIP,
                  "deposition scratch allocation failed");
    }
  }
  hipError_t e = deposit_run(D, Lo, ctx->dep_buf, s, ctx->dep_flag_h, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "pcol_deposit");
  if (st != PCOL_OK) return fail(ctx, st, "position outside [0, L) or not finite");
  return PCOL_OK;
}

pcol_status pcol_deposit_noalloc(const double *x, const double *y, const double *z, int64_t n,
                                 const double *a, int comp, const int32_t nc[3],
                                 const double len[3], double *out, void *hip_stream) {
  DepositArgs D{};
  const char *why = nullptr;
  pcol_status st = deposit_args(x, y, z, n, a, comp, nc, len, out, D, why);
  if (st != PCOL_OK) return st;
  const DepositLayout Lo = deposit_layout(D.n, D.nnode, comp);
  if (Lo.bytes > (int64_t)PCOL_NOALLOC_SCRATCH_BYTES) return PCOL_E_SCRATCH;
  unsigned char *base = nullptr;
  if (static_scratch(&base) != hipSuccess) return PCOL_E_HIP;
  unsigned int flag_h = 0u;  // pageable host word: no pinned allocation
  if (deposit_run(D, Lo, base, (hipStream_t)hip_stream, &flag_h, st) != hipSuccess)
    return PCOL_E_HIP;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------- batched form

namespace {

BatchDev batch_dev(const BatchPlan *bp) {
  BatchDev B{};
  B.gtab = bp->gtab;
  B.cell_base = bp->cell_base;
  B.box_of = bp->box_of;
  B.box_off = bp->box_off_d;
  B.breach = bp->breach;
  B.nchunk = bp->nchunk;
  B.chunk_box = bp->chunk_box;
  B.chunk_lo = bp->chunk_lo;
  B.bmax = bp->bmax;
  B.flags = bp->flags;
  B.nbox = bp->nbox;
  return B;
}

// Grid of one box: cell side >= reach * mult * 1.05 per axis (the slack lets
// the reach grow a little over later steps before a re-plan), no more cells
// than max(27, n_b / 8) for a box of n_b spheres (sparse boxes get cells of
// about 8 spheres: the per-cell work of the pair tests outweighs the extra
// pairs), and at least 3 cells per axis (else the box is rejected).
bool box_grid(const double len[3], int64_t nb, double reach, double mult, Grid &G) {
  double cell = reach * mult * 1.05;
  const double vol = len[0] * len[1] * len[2];
  const double most = (double)nb / 8.0 > 27.0 ? (double)nb / 8.0 : 27.0;
  const double floor_side = cbrt(vol / most);
  if (!(cell >= floor_side)) cell = floor_side;
  for (int a = 0; a < 3; ++a) {
    double q = floor(len[a] / (cell * (1.0 + 1e-9)));
    if (q > 1024.0) q = 1024.0;
    if (q < 3.0) {
      // fall back to exactly 3 cells when they are still at least the reach wide
      if (len[a] / 3.0 >= reach * (1.0 + 1e-9))
        q = 3.0;
      else
        return false;
    }
    G.nc[a] = (int)q;
    G.L[a] = len[a];
    G.halfL[a] = 0.5 * len[a];
    G.sL[a] = len[a];
    G.inv_h[a] = q / len[a];
    G.h[a] = len[a] / q;
  }
  G.ncell = G.nc[0] * G.nc[1] * G.nc[2];
  G.inv_row = 1.0 / G.nc[0];
  G.inv_layer = 1.0 / ((double)G.nc[0] * G.nc[1]);
  return true;
}

template <typename T>
hipError_t regrow(T **p, int64_t want) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  return hipMalloc((void **)p, (size_t)(want > 0 ? want : 1) * sizeof(T));
}

// read back the flags and totals of the last batched run
hipError_t batch_readback(pcol_ctx *ctx, BatchPlan *bp) {
  hipError_t e = hipMemcpyAsync(bp->flags_h, bp->flags, 16 * sizeof(unsigned int),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(bp->flags_h + 16, bp->totals, 3 * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e;
}

unsigned long long batch_total(const BatchPlan *bp, int k) {
  unsigned long long v;
  memcpy(&v, (const char *)(bp->flags_h + 16) + 8 * k, 8);
  return v;
}

}  // namespace

// (Re)build the per-box tables for this layout and the current data: per-box
// reach on the device, then grids and cell numbering on the host.
static pcol_status batch_plan(pcol_ctx *ctx, int nbox, const int64_t *box_off,
                              const pcol_box *boxes, const Particles &P, double dt, double mult) {
  BatchPlan *bp = ctx->bp;
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  if (nbox > bp->cap_box) {
    if ((e = regrow(&bp->gtab, nbox)) != hipSuccess ||
        (e = regrow(&bp->cell_base, nbox + 1)) != hipSuccess ||
        (e = regrow(&bp->box_off_d, nbox + 1)) != hipSuccess ||
        (e = regrow(&bp->breach, nbox)) != hipSuccess ||
        (e = regrow(&bp->bmax, nbox)) != hipSuccess)
      return fail(ctx, PCOL_E_NOMEM, "batched tables");
    bp->cap_box = nbox;
  }
  // chunks of the reach pass: each box cut into pieces of BREACH_CHUNK spheres
  std::vector<int> &cbox = bp->chunk_box_h;
  std::vector<int64_t> &clo = bp->chunk_lo_h;
  cbox.clear();
  clo.clear();
  for (int b = 0; b < nbox; ++b)
    for (int64_t lo = box_off[b]; lo < box_off[b + 1]; lo += BREACH_CHUNK) {
      cbox.push_back(b);
      clo.push_back(lo);
    }
  if ((int)cbox.size() > bp->cap_chunk) {
    if ((e = regrow(&bp->chunk_box, (int64_t)cbox.size())) != hipSuccess ||
        (e = regrow(&bp->chunk_lo, (int64_t)cbox.size())) != hipSuccess)
      return fail(ctx, PCOL_E_NOMEM, "batched tables");
    bp->cap_chunk = (int)cbox.size();
  }
  bp->nchunk = (int)cbox.size();
  if (!cbox.empty()) {
    PCOL_HIP(hipMemcpyAsync(bp->chunk_box, cbox.data(), cbox.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    PCOL_HIP(hipMemcpyAsync(bp->chunk_lo, clo.data(), clo.size() * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  }
  PCOL_HIP(hipMemsetAsync(bp->bmax, 0, (size_t)nbox * sizeof(BoxMax), s));
  if (P.n > bp->cap_n) {
    if ((e = regrow(&bp->box_of, P.n)) != hipSuccess)
      return fail(ctx, PCOL_E_NOMEM, "batched tables");
    bp->cap_n = P.n;
  }
  if (!bp->flags) {
    if (hipMalloc((void **)&bp->flags, 16 * sizeof(unsigned int)) != hipSuccess ||
        hipMalloc((void **)&bp->totals, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&bp->flags_h, 16 * sizeof(unsigned int) + 4 * 8) != hipSuccess)
      return fail(ctx, PCOL_E_NOMEM, "batched flags");
  }
  bp->nbox = nbox;
  bp->n = P.n;
  bp->box_off.assign(box_off, box_off + nbox + 1);
  bp->len.resize((size_t)3 * nbox);
  bp->gtab_h.assign(nbox, Grid{});
  for (int b = 0; b < nbox; ++b)
    for (int a = 0; a < 3; ++a) {
      bp->len[3 * b + a] = boxes[b].len[a];
      bp->gtab_h[b].L[a] = boxes[b].len[a];
      bp->gtab_h[b].nc[a] = 1;
    }
  PCOL_HIP(hipMemcpyAsync(bp->box_off_d, box_off, (nbox + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  PCOL_HIP(hipMemcpyAsync(bp->gtab, bp->gtab_h.data(), nbox * sizeof(Grid), hipMemcpyHostToDevice, s));
  PCOL_HIP(launch_fill_box_of(s, nbox, bp->box_off_d, bp->box_of));
  PCOL_HIP(launch_fill_u32(s, bp->flags, 0u, 16));
  PCOL_HIP(launch_breach(s, P, batch_dev(bp), dt, 0));
  bp->breach_h.resize(nbox);
  PCOL_HIP(hipMemcpyAsync(bp->breach_h.data(), bp->breach, nbox * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  PCOL_HIP(batch_readback(ctx, bp));
  const unsigned int err = bp->flags_h[FLAG_ERR];
  if (err & ERR_INVALID) return fail(ctx, PCOL_E_INVALID, "non-finite value, r <= 0, m <= 0 or position outside its box");
  if (err & ERR_BOX) return fail(ctx, PCOL_E_BOX, "a box side <= 2 * reach");
  bp->cell_base_h.assign(nbox + 1, 0);
  int64_t total = 0;
  for (int b = 0; b < nbox; ++b) {
    double len[3] = {boxes[b].len[0], boxes[b].len[1], boxes[b].len[2]};
    if (!box_grid(len, box_off[b + 1] - box_off[b], bp->breach_h[b], mult, bp->gtab_h[b]))
      return fail(ctx, PCOL_E_BOX, "batched form needs 3 cells of at least the reach per axis");
    bp->cell_base_h[b] = (int)total;
    total += bp->gtab_h[b].ncell;
    if (total > (1 << 28)) return fail(ctx, PCOL_E_BOX, "too many cells in the batch");
  }
  bp->cell_base_h[nbox] = (int)total;
  bp->total_cells = (int)total;
  PCOL_HIP(hipMemcpyAsync(bp->gtab, bp->gtab_h.data(), nbox * sizeof(Grid), hipMemcpyHostToDevice, s));
  PCOL_HIP(hipMemcpyAsync(bp->cell_base, bp->cell_base_h.data(), (nbox + 1) * sizeof(int),
                          hipMemcpyHostToDevice, s));
  if (total + 2 > ctx->cell_cap) {
    if (ctx->count) (void)hipFree(ctx->count);
    if (ctx->start) (void)hipFree(ctx->start);
    if (ctx->blocksum) (void)hipFree(ctx->blocksum);
    ctx->count = ctx->start = ctx->blocksum = nullptr;
    ctx->cell_cap = 0;
    const int64_t cap = total + 2;
    hipError_t a = dalloc(&ctx->count, (size_t)cap);
    if (a == hipSuccess) a = dalloc(&ctx->start, (size_t)cap + 1);
    if (a == hipSuccess) a = dalloc(&ctx->blocksum, (size_t)(cap / 4096 + 2));
    if (a != hipSuccess) return fail(ctx, PCOL_E_NOMEM, "cell arrays");
    ctx->cell_cap = cap;
  }
  PCOL_HIP(hipStreamSynchronize(s));
  bp->tables = true;
  bp->cell_mult = mult;
  return PCOL_OK;
}

// Enqueue the whole batched step on stream s (captured into a graph).
static pcol_status batch_enqueue(pcol_ctx *ctx, hipStream_t s, const Particles &P, int32_t *part,
                                 double *tc, double dt, double e, int kmax, int cpw) {
  BatchPlan *bp = ctx->bp;
  const BatchDev B = batch_dev(bp);
  const int n = (int)P.n;
  const int ncell = bp->total_cells;
  PCOL_HIP(launch_fill_u32(s, bp->flags, 0u, 16));
  PCOL_HIP(launch_fill_u32(s, (unsigned int *)bp->totals, 0u, 8));
  PCOL_HIP(launch_fill_u32(s, (unsigned int *)ctx->ctr_d, 0u, sizeof(SweepCounters) / 4));
  // reach check and cell ids in one pass over the spheres (the counts are
  // discarded with everything else if the check fails)
  PCOL_HIP(launch_fill_i32(s, ctx->count, 0, ncell));
  PCOL_HIP(launch_breach(s, P, B, dt, 1, ctx->cid, ctx->slot, ctx->count));
  PCOL_HIP(launch_scan(s, ctx->count, ncell, ctx->start, ctx->blocksum, ctx->reach_d));
  PCOL_HIP(launch_scatter(s, P, ctx->cid, ctx->slot, ctx->start, ctx->rec, ctx->rank, &B));
  PCOL_HIP(launch_fill_u8(s, ctx->status, ST_ACTIVE, n));
  PCOL_HIP(launch_fill_i32(s, ctx->cnt, 0, n));
  DetectArgs A{};
  A.rec = ctx->rec;
  A.start = ctx->start;
  A.cnt = ctx->cnt;
  A.slot_t = ctx->slot_t;
  A.slot_j = ctx->slot_j;
  A.ctr = ctx->ctr_d;
  A.n = n;
  A.dt = dt;
  A.dt2 = 2.0 * dt * (1.0 + 0x1.0p-20);
  // Filter tolerance (see the single-box detect) from bounds that hold for any
  // data the graph accepts: the re-plan check stops the step unless every
  // box's reach 2 rmax + 2 vmax dt is at most its cell side, so with hmax the
  // largest cell side, reach <= hmax, 2 rmax <= hmax and 2 vmax <= hmax / dt.
  double hmax = 0.0;
  for (const Grid &G : bp->gtab_h)
    for (int a = 0; a < 3; ++a) hmax = G.h[a] > hmax ? G.h[a] : hmax;
  A.tol = 16.0 * 0x1.0p-53 * hmax * hmax * (2.0 + A.dt2 / dt);
  {
    // reach <= hmax, 2 r_max <= hmax and 2 v_max dt <= hmax in every box (see above)
    double Lmax = 0.0;
    for (const Grid &G : bp->gtab_h)
      for (int a = 0; a < 3; ++a) Lmax = G.L[a] > Lmax ? G.L[a] : Lmax;
    A.tol64 = gram64_tolerance(hmax, hmax, hmax / (2.0 * dt), 0.5 * hmax, Lmax, A.dt2);
  }
  A.K = ctx->K;
  A.fp32 = 0;
  PCOL_HIP(launch_detect_batched(s, A, B, bp->total_cells, cpw));
  PCOL_HIP(launch_slot_min(s, n, 1, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                           ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d, bp->flags));
  PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec, ctx->start,
                               ctx->G, dt, ctx->status, ctx->key_j, ctx->key_t, &B));
  for (int k = 0; k < kmax; ++k) {
    PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, P.m, ctx->key_j, ctx->key_t,
                                  ctx->status, ctx->out, ctx->ctr_d, &B));
    PCOL_HIP(launch_sweep_check(s, ctx->ctr_d, bp->flags, bp->totals, k == kmax - 1));
    PCOL_HIP(launch_slot_min(s, n, 0, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                             ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d, bp->flags));
    PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec,
                                 ctx->start, ctx->G, dt, ctx->status, ctx->key_j,
                                 ctx->key_t, &B));
  }
  PCOL_HIP(launch_finish(s, P, ctx->rank, ctx->out, ctx->status, part, tc, dt, ctx->G,
                         &B));
  return PCOL_OK;
}

static pcol_status batch_capture(pcol_ctx *ctx, const Particles &P, int32_t *part, double *tc,
                                 double dt, double e, int kmax, int cpw, hipGraphExec_t *exec) {
  BatchPlan *bp = ctx->bp;
  if (!bp->gstream) PCOL_HIP(hipStreamCreateWithFlags(&bp->gstream, hipStreamNonBlocking));
  PCOL_HIP(hipStreamBeginCapture(bp->gstream, hipStreamCaptureModeRelaxed));
  pcol_status st = batch_enqueue(ctx, bp->gstream, P, part, tc, dt, e, kmax, cpw);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(bp->gstream, &g);
  if (st != PCOL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ee != hipSuccess) return hip_fail(ctx, ee, "hipStreamEndCapture");
  ee = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ee != hipSuccess) return hip_fail(ctx, ee, "hipGraphInstantiate");
  return PCOL_OK;
}

// Finish a step whose captured sweeps ran out: remaining sweeps on the host
// loop, then free flight and the copy back (the graph skipped both).
static pcol_status batch_finish(pcol_ctx *ctx, const Particles &P, int32_t *part, double *tc,
                                double dt, double e, int64_t &pairs, int64_t &sweeps) {
  BatchPlan *bp = ctx->bp;
  const BatchDev B = batch_dev(bp);
  hipStream_t s = ctx->stream;
  const int n = (int)P.n;
  for (;;) {
    PCOL_HIP(launch_fill_u32(s, (unsigned int *)ctx->ctr_d, 0u, sizeof(SweepCounters) / 4));
    PCOL_HIP(launch_resolve_sweep(s, n, ctx->rec, ctx->G, dt, e, P.m, ctx->key_j, ctx->key_t,
                                  ctx->status, ctx->out, ctx->ctr_d, &B));
    PCOL_HIP(hipMemcpyAsync(ctx->ctr_h, ctx->ctr_d, sizeof(SweepCounters), hipMemcpyDeviceToHost, s));
    PCOL_HIP(hipStreamSynchronize(s));
    unsigned long long sp, sc;
    sum_counters(*ctx->ctr_h, sp, sc);
    ++sweeps;
    pairs += (int64_t)sp;
    if (sp == 0ull) break;
    PCOL_HIP(launch_fill_u32(s, (unsigned int *)ctx->ctr_d, 0u, sizeof(SweepCounters) / 4));
    PCOL_HIP(launch_slot_min(s, n, 0, ctx->cnt, ctx->slot_t, ctx->slot_j, ctx->K, ctx->status,
                             ctx->rec, ctx->key_j, ctx->key_t, ctx->ovf, ctx->ctr_d, bp->flags));
    PCOL_HIP(launch_gather_exact(s, ctx->ovf, 0, &ctx->ctr_d->n_overflow, -1, ctx->rec,
                                 ctx->start, ctx->G, dt, ctx->status, ctx->key_j,
                                 ctx->key_t, &B));
  }
  PCOL_HIP(launch_fill_u32(s, bp->flags + FLAG_UNFINISHED, 0u, 1));
  PCOL_HIP(launch_finish(s, P, ctx->rank, ctx->out, ctx->status, part, tc, dt, ctx->G,
                         &B));
  return PCOL_OK;
}

static std::string tune_key(int nbox, int64_t n, const int64_t *box_off, const pcol_box *boxes,
                            double dt) {
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  double vol = 0.0;
  for (int b = 0; b < nbox; ++b) vol += boxes[b].len[0] * boxes[b].len[1] * boxes[b].len[2];
  std::ostringstream k;
  k << "c" << prop.gcnArchName << "|n" << (int)round(log2((double)(n > 0 ? n : 1))) << "|b"
    << (int)round(log2((double)nbox)) << "|rho" << (int)round(4.0 * log2(n / vol + 1e-300))
    << "|dt" << dt;
  (void)box_off;
  std::string key = k.str();
  for (char &c : key)
    if (c == ' ') c = '_';
  return key;
}

static std::string tune_path() {
  const char *p = getenv("PCOL_TUNE_CACHE");
  if (p && *p) return p;
  const char *h = getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/pcol_tune.txt";
}

static bool tune_lookup(const std::string &key, double &mult, int &cpw) {
  std::ifstream f(tune_path());
  std::string k;
  double m;
  int w;
  bool found = false;
  while (f >> k >> m >> w)
    if (k == key) {
      mult = m;
      cpw = w;
      found = true;
    }
  return found;
}

static void tune_store(const std::string &key, double mult, int cpw) {
  std::ofstream f(tune_path(), std::ios::app);
  if (f) f << key << " " << mult << " " << cpw << "\n";
}

// Time candidate (cell size factor, home cells per workgroup) pairs on scratch
// copies of the input; keep the fastest.  Every candidate computes the same
// step (the result does not depend on the cell size or the launch shape).
static pcol_status batch_autotune(pcol_ctx *ctx, int nbox, const int64_t *box_off,
                                  const pcol_box *boxes, const Particles &P, double dt,
                                  double e) {
  BatchPlan *bp = ctx->bp;
  hipStream_t s = ctx->stream;
  const int64_t n = P.n;
  if (bp->tune_cap < n) {
    if (bp->tune_buf) (void)hipFree(bp->tune_buf);
    bp->tune_buf = nullptr;
    if (hipMalloc((void **)&bp->tune_buf, (size_t)(n > 0 ? n : 1) * 6 * sizeof(double)) != hipSuccess)
      return fail(ctx, PCOL_E_NOMEM, "tuning scratch");
    bp->tune_cap = n;
  }
  Particles T = P;
  double *src[6] = {P.x, P.y, P.z, P.vx, P.vy, P.vz};
  double *dst[6];
  for (int k = 0; k < 6; ++k) dst[k] = bp->tune_buf + (size_t)k * n;
  T.x = dst[0];
  T.y = dst[1];
  T.z = dst[2];
  T.vx = dst[3];
  T.vy = dst[4];
  T.vz = dst[5];
  const double mults[3] = {1.0, 1.15, 1.3};
  const int shapes[3] = {2, 4, 8};  // home cells per workgroup
  double best = 1e300, best_mult = 1.0;
  int best_cpw = 4;
  for (double mult : mults) {
    pcol_status st = batch_plan(ctx, nbox, box_off, boxes, P, dt, mult);
    if (st == PCOL_E_BOX) continue;  // this cell size leaves some box under 3 cells
    if (st != PCOL_OK) return st;
    for (int cpw : shapes) {
      hipGraphExec_t ex = nullptr;
      if ((st = batch_capture(ctx, T, ctx->partner_tmp, ctx->tcoll_tmp, dt, e, bp->kmax, cpw,
                              &ex)) != PCOL_OK)
        return st;
      float times[3];
      for (int rep = 0; rep < 3; ++rep) {
        for (int k = 0; k < 6; ++k)
          PCOL_HIP(hipMemcpyAsync(dst[k], src[k], n * sizeof(double), hipMemcpyDeviceToDevice, s));
        PCOL_HIP(hipEventRecord(ctx->ev[0], s));
        PCOL_HIP(hipGraphLaunch(ex, s));
        PCOL_HIP(hipEventRecord(ctx->ev[1], s));
        PCOL_HIP(hipEventSynchronize(ctx->ev[1]));
        (void)hipEventElapsedTime(&times[rep], ctx->ev[0], ctx->ev[1]);
      }
      (void)hipGraphExecDestroy(ex);
      std::sort(times, times + 3);
      if (times[1] < best) {
        best = times[1];
        best_mult = mult;
        best_cpw = cpw;
      }
    }
  }
  bp->cell_mult = best_mult;
  bp->cpw = best_cpw;
  bp->tuned = true;
  bp->tables = false;
  return PCOL_OK;
}

extern "C" pcol_status pcol_step_batched(pcol_ctx *ctx, int32_t nbox, const int64_t *box_off,
                                         const pcol_box *boxes, pcol_particles *p, double dt,
                                         double e, int32_t *partner, double *tcoll,
                                         pcol_batch_stats *stats) {
  if (!ctx) return PCOL_E_INVALID;
  if (ctx->opts.order == 1)
    return fail(ctx, PCOL_E_INVALID, "the literal order (opts.order = 1) is built for pcol_step only");
  if (nbox < 1 || !box_off || !boxes || !p) return fail(ctx, PCOL_E_INVALID, "bad batch arguments");
  pcol_box any{{1.0, 1.0, 1.0}};
  pcol_status st = check_common(ctx, p, &any, dt);
  if (st != PCOL_OK) return st;
  if (!(e >= 0.0 && e <= 1.0)) return fail(ctx, PCOL_E_INVALID, "e outside [0, 1]");
  if (box_off[0] != 0 || box_off[nbox] != p->n)
    return fail(ctx, PCOL_E_INVALID, "box_off must run from 0 to n");
  for (int b = 0; b < nbox; ++b) {
    if (box_off[b + 1] < box_off[b]) return fail(ctx, PCOL_E_INVALID, "box_off not increasing");
    for (int a = 0; a < 3; ++a)
      if (!finite_pos(boxes[b].len[a])) return fail(ctx, PCOL_E_INVALID, "box side not finite positive");
  }
  if (!ctx->bp) {
    ctx->bp = new (std::nothrow) BatchPlan();
    if (!ctx->bp) return PCOL_E_NOMEM;
    if (ctx->opts.max_sweeps > 0) ctx->bp->kmax = ctx->opts.max_sweeps;
  }
  BatchPlan *bp = ctx->bp;
  const Particles P = to_dev(p);
  int32_t *part = partner ? partner : ctx->partner_tmp;
  double *tc = tcoll ? tcoll : ctx->tcoll_tmp;
  const void *ptrs[8] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->r, p->m};
  bool same_layout = bp->tables && bp->nbox == nbox && bp->n == p->n &&
                     std::equal(box_off, box_off + nbox + 1, bp->box_off.begin());
  for (int b = 0; same_layout && b < nbox; ++b)
    for (int a = 0; a < 3; ++a)
      if (bp->len[3 * b + a] != boxes[b].len[a]) same_layout = false;
  int replanned = 0, tuned = 0, host_finish = 0;
  if (!same_layout && !bp->tuned && ctx->opts.autotune) {
    const std::string key = tune_key(nbox, p->n, box_off, boxes, dt);
    double m;
    int w;
    if (tune_lookup(key, m, w)) {
      bp->cell_mult = m;
      bp->cpw = w;
      bp->tuned = true;
    } else {
      if ((st = batch_autotune(ctx, nbox, box_off, boxes, P, dt, e)) != PCOL_OK) return st;
      tune_store(key, bp->cell_mult, bp->cpw);
      tuned = 1;
    }
  }
  if (!ctx->opts.autotune && !bp->tuned) {
    bp->cell_mult = ctx->opts.cell_mult;
    bp->cpw = 4;
  }
  for (int attempt = 0;; ++attempt) {
    if (!same_layout || !bp->tables) {
      if ((st = batch_plan(ctx, nbox, box_off, boxes, P, dt, bp->cell_mult)) != PCOL_OK) return st;
      same_layout = true;
      bp->captured = false;
      replanned = 1;
    }
    bool recapture = !bp->captured || bp->cap_dt != dt || bp->cap_e != e || bp->cap_part != part ||
                     bp->cap_tc != tc;
    for (int k = 0; k < 8 && !recapture; ++k) recapture = bp->cap_ptr[k] != ptrs[k];
    if (recapture) {
      if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
      bp->exec = nullptr;
      if ((st = batch_capture(ctx, P, part, tc, dt, e, bp->kmax, bp->cpw, &bp->exec)) != PCOL_OK)
        return st;
      bp->captured = true;
      bp->cap_dt = dt;
      bp->cap_e = e;
      bp->cap_part = part;
      bp->cap_tc = tc;
      for (int k = 0; k < 8; ++k) bp->cap_ptr[k] = ptrs[k];
    }
    PCOL_HIP(hipGraphLaunch(bp->exec, ctx->stream));
    PCOL_HIP(batch_readback(ctx, bp));
    const unsigned int err = bp->flags_h[FLAG_ERR];
    if (err & ERR_INVALID)
      return fail(ctx, PCOL_E_INVALID, "non-finite value, r <= 0, m <= 0 or position outside its box");
    if (err & ERR_BOX) return fail(ctx, PCOL_E_BOX, "a box side <= 2 * reach");
    if (err & ERR_REPLAN) {  // reach outgrew the planned cells; nothing was written
      if (attempt > 0) return fail(ctx, PCOL_E_HIP, "batched re-plan did not settle");
      bp->tables = false;
      continue;
    }
    break;
  }
  int64_t pairs = (int64_t)batch_total(bp, 0);
  int64_t sweeps = bp->flags_h[FLAG_SWEEPS];
  if (bp->flags_h[FLAG_UNFINISHED]) {
    if ((st = batch_finish(ctx, P, part, tc, dt, e, pairs, sweeps)) != PCOL_OK) return st;
    PCOL_HIP(hipStreamSynchronize(ctx->stream));
    host_finish = 1;
    if (ctx->opts.max_sweeps == 0) {  // capture enough sweeps next time
      bp->kmax = (int)sweeps + 4;
      bp->captured = false;
    }
  } else if (ctx->opts.max_sweeps == 0 && bp->kmax > (int)sweeps + 4) {
    // far more sweep slots than the step used: each empty slot still launches
    // its kernels (early exits, about 25 us a slot), so capture fewer next time,
    // keeping room for two more sweeps than this step took
    bp->kmax = (int)sweeps + 2;
    bp->captured = false;
  }
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_pairs = pairs;
    stats->n_sweeps = sweeps;
    stats->contacts = (int64_t)(batch_total(bp, 1) / 2ull);
    stats->n_overflow = (int64_t)batch_total(bp, 2);
    stats->total_cells = bp->total_cells;
    stats->replanned = replanned;
    stats->finished_on_host = host_finish;
    stats->tuned = tuned;
    stats->home_cells = bp->cpw;
    stats->cell_mult = bp->cell_mult;
  }
  return PCOL_OK;
}
