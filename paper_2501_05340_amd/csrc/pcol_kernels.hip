// HIP kernels of the pcol collision step (gfx950, wave64).  Each kernel states
// the step of the method it implements; the rule numbers refer to the header
// comment of include/pcol.h.
#include "pcol_internal.h"

#include <math.h>

#include <algorithm>

namespace pcol {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// Exclusive position of this lane among the lanes of the wave for which `pred`
// holds, and one atomic per wave on `counter` for all of them.  Returns the
// slot of this lane (valid only where pred).
__device__ __forceinline__ unsigned int wave_append(bool pred, unsigned int *counter) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return 0u;
  const unsigned int lane = __lane_id();
  const unsigned int below = __popcll(mask & ((1ull << lane) - 1ull));
  const int leader = __ffsll((long long)mask) - 1;
  unsigned int base = 0u;
  if ((int)lane == leader) base = atomicAdd(counter, (unsigned int)__popcll(mask));
  base = __shfl(base, leader);
  return base + below;
}

// Slot of this lane's key among all items of that key (key < 0: none, returns
// 0): consecutive lanes with one key (inputs stored in key order) share one
// atomic on count[key] per run and take consecutive slots.  Every lane of the
// wave must call it.
__device__ __forceinline__ int run_slot(int key, int *count) {
  const int lane = (int)__lane_id();
  const int prev = __shfl_up(key, 1);
  const unsigned long long starts = __ballot(lane == 0 || prev != key);
  const unsigned long long upto = starts & ((2ull << lane) - 1ull);  // bit 0 always set
  const int h = 63 - __clzll(upto);                                   // this lane's run start
  const unsigned long long after = starts & ~((2ull << lane) - 1ull);
  int base = 0;
  if (key >= 0 && lane == h) {
    const int len = (after ? __ffsll((long long)after) - 1 : WAVE) - h;
    base = atomicAdd(&count[key], len);
  }
  return __shfl(base, h) + (lane - h);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// blockIdx -> logical block so that each of the 8 XCDs (which receive
// workgroups round-robin) walks one contiguous range of logical blocks: spatial
// neighbours then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int x = bid % 8;
  return x * q + (x < r ? x : r) + bid / 8;
}

// Sum of v over the workgroup added to *target by one atomic (blockDim a
// multiple of the wave size, at most 1024 threads).
__device__ __forceinline__ void block_add(unsigned long long v, unsigned long long *target) {
  __shared__ unsigned long long part[1024 / WAVE];
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  if (__lane_id() == 0) part[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0ull;
    for (int k = 0; k < nw; ++k) tot += part[k];
    if (tot) atomicAdd(target, tot);
  }
  __syncthreads();
}

__device__ __forceinline__ CounterShard &my_shard(SweepCounters *ctr) {
  return ctr->shard[blockIdx.x % NSHARD];
}

}  // namespace

// ---------------------------------------------------------------- fills

__global__ void k_fill_u32(unsigned int *p, unsigned int v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static int fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : (int)g;
}

hipError_t launch_fill_u32(hipStream_t s, unsigned int *p, unsigned int v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(hipStream_t s, int *p, int v, int64_t n) {
  return launch_fill_u32(s, (unsigned int *)p, (unsigned int)v, n);
}
hipError_t launch_fill_u8(hipStream_t s, uint8_t *p, uint8_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(hipStream_t s, double *p, double v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a1: reach + validation

// Largest |v|^2, radius and extent r + |v| dt, smallest radius, data validity,
// and the histogram of extents (Sec. "Collision Operator": the halo must hold
// every partner a sphere can reach within the step).  The maxima and the
// validity cover every sphere; the histogram, which only picks the split
// extent (a performance choice), covers the spheres whose index is a multiple
// of 2^hist_shift.  Grid-stride over at most REACH_BLOCKS workgroups; each
// histograms in LDS and stores its partial results (maxima and its whole
// histogram) in parts, which k_reach_final reduces: no address takes an atomic
// from every workgroup.
// BIN: the same pass also takes each sphere's cell and slot on the grid G with
// split extent rho_c, exactly as k_cell_hist does (the binning of a step whose
// grid is planned before its reach is known; the plan is checked against the
// reach afterwards).  A sphere that fails the checks still gets a cell inside
// the grid, and the caller discards the pass.
template <bool BIN>
__global__ __launch_bounds__(256) void k_reach(Particles P, double L0, double L1, double L2,
                                               double dt, int hist_shift, ReachPart *parts,
                                               unsigned int *phist, Grid G, double rho_c,
                                               int *cid, int *slot, int *count) {
  __shared__ unsigned int hist[RHO_BINS];
  for (int k = threadIdx.x; k < RHO_BINS; k += 256) hist[k] = 0u;
  __syncthreads();
  double v2 = 0.0, rm = 0.0, rn = INFINITY, em = 0.0;
  unsigned int bad = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t hmask = ((int64_t)1 << hist_shift) - 1;
  // four elements per thread per step: their loads are issued together.  The
  // loop runs while the wave's first element is in range, so that every lane
  // of a wave takes each step (the binning's run_slot needs the whole wave);
  // lanes past the end hold no element.
  const int64_t wbase = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(WAVE - 1));
  for (int64_t w0 = wbase; w0 < P.n; w0 += 4 * stride) {
    const int64_t i0 = w0 + (threadIdx.x & (WAVE - 1));
    double x[4], y[4], z[4], vx[4], vy[4], vz[4], r[4], m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < P.n) {
        x[u] = P.x[i];
        y[u] = P.y[i];
        z[u] = P.z[i];
        vx[u] = P.vx[i];
        vy[u] = P.vy[i];
        vz[u] = P.vz[i];
        r[u] = P.r[i];
        m[u] = P.m[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = i0 + u * stride < P.n;
      bool has = false;
      int bin = -1;
      if (in) {
        const double w = (vx[u] * vx[u] + vy[u] * vy[u]) + vz[u] * vz[u];
        const bool fin = isfinite(x[u]) && isfinite(y[u]) && isfinite(z[u]) && isfinite(w) &&
                         isfinite(r[u]) && isfinite(m[u]);
        if (!fin || !(r[u] > 0.0) || !(m[u] > 0.0)) bad |= 1u;
        if (P.wx) {
          const int64_t i = i0 + u * stride;
          if (!isfinite(P.wx[i]) || !isfinite(P.wy[i]) || !isfinite(P.wz[i])) bad |= 1u;
        }
        if (!(x[u] >= 0.0 && x[u] < L0) || !(y[u] >= 0.0 && y[u] < L1) ||
            !(z[u] >= 0.0 && z[u] < L2))
          bad |= 2u;
        if (fin) {
          v2 = w > v2 ? w : v2;
          rm = r[u] > rm ? r[u] : rm;
          rn = r[u] < rn ? r[u] : rn;
          if (r[u] > 0.0) {
            const double ex = extent(r[u], vx[u], vy[u], vz[u], dt);
            em = ex > em ? ex : em;
            has = ((i0 + u * stride) & hmask) == 0;
            if (has) bin = rho_bin(ex);  // -1 (no lane's bin) for the others
          }
        }
      }
      if (BIN) {  // the cell and slot (every lane of the wave takes part)
        int c = -1;
        if (in) {
          const int cx = cell_coord(x[u], G.inv_h[0], G.nc[0]);
          const int cy = cell_coord(y[u], G.inv_h[1], G.nc[1]);
          const int cz = cell_coord(z[u], G.inv_h[2], G.nc[2]);
          c = (cz * G.nc[1] + cy) * G.nc[0] + cx;
          if (G.layer2 && !(extent(r[u], vx[u], vy[u], vz[u], dt) <= rho_c)) c += G.layer2;
        }
        const int sl = run_slot(c, count);
        if (c >= 0) {
          cid[i0 + u * stride] = c;
          slot[i0 + u * stride] = sl;
        }
      }
      // histogram: one LDS atomic per distinct bin of the wave (lanes of one
      // bin add together), so the few busy bins see no lane conflicts
      unsigned long long todo = __ballot(has);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __shfl(bin, leader);
        const unsigned long long same = __ballot(bin == lb);
        if ((int)__lane_id() == leader) atomicAdd(&hist[lb], (unsigned int)__popcll(same));
        todo &= ~same;
      }
    }
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double a = __shfl_xor(v2, o), b = __shfl_xor(rm, o), c = __shfl_xor(rn, o),
                 d = __shfl_xor(em, o);
    v2 = a > v2 ? a : v2;
    rm = b > rm ? b : rm;
    rn = c < rn ? c : rn;
    em = d > em ? d : em;
    bad |= __shfl_xor(bad, o);
  }
  __shared__ ReachPart wpart[256 / WAVE];
  if (__lane_id() == 0)
    wpart[threadIdx.x / WAVE] = ReachPart{dbits(v2), dbits(rm), dbits(rn), dbits(em), bad, 0u};
  __syncthreads();
  if (threadIdx.x == 0) {
    ReachPart p = wpart[0];
    for (int w = 1; w < 256 / WAVE; ++w) p = reach_merge(p, wpart[w]);
    parts[blockIdx.x] = p;
  }
  for (int k = threadIdx.x; k < RHO_BINS; k += 256)
    phist[(int64_t)blockIdx.x * RHO_BINS + k] = hist[k];
}

// Reduction of k_reach's nblocks partial results into out: the maxima, the
// smallest radius and the validity bits by one workgroup, the histogram by
// REACH_FINAL_Y workgroups per 256 bins, each summing a share of the partial
// histograms and adding its non-zero sums (REACH_FINAL_Y adds per bin at most).
constexpr int REACH_FINAL_Y = 32;

__global__ __launch_bounds__(256) void k_reach_final(int nblocks, const ReachPart *parts,
                                                     const unsigned int *phist, ReachOut *out) {
  const int b = blockIdx.x * 256 + threadIdx.x;  // bin
  const int per = (nblocks + REACH_FINAL_Y - 1) / REACH_FINAL_Y;
  const int k0 = blockIdx.y * per, k1 = k0 + per < nblocks ? k0 + per : nblocks;
  unsigned int s = 0u;
  for (int k = k0; k < k1; ++k) s += phist[(int64_t)k * RHO_BINS + b];
  if (s) atomicAdd(&out->hist[b], s);
  if (blockIdx.x != 0 || blockIdx.y != 0) return;
  __shared__ ReachPart red[256];
  ReachPart p{0ull, 0ull, dbits(INFINITY), 0ull, 0u, 0u};
  for (int k = threadIdx.x; k < nblocks; k += 256) p = reach_merge(p, parts[k]);
  red[threadIdx.x] = p;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = reach_merge(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out->v2max = red[0].v2max;
    out->rmax = red[0].rmax;
    out->rhomax = red[0].rhomax;
    out->rmin = red[0].rmin;
    out->bad = red[0].bad;
  }
}

hipError_t launch_reach(hipStream_t s, const Particles &P, const double L[3], double dt,
                        int hist_shift, ReachOut *out, ReachPart *parts, unsigned int *phist,
                        const Grid *G, double rho_c, int *cid, int *slot, int *count) {
  int64_t g = (P.n + 255) / 256;
  if (g > REACH_BLOCKS) g = REACH_BLOCKS;
  if (g < 1) g = 1;
  if (G)
    hipLaunchKernelGGL(k_reach<true>, dim3((int)g), dim3(256), 0, s, P, L[0], L[1], L[2], dt,
                       hist_shift, parts, phist, *G, rho_c, cid, slot, count);
  else
    hipLaunchKernelGGL(k_reach<false>, dim3((int)g), dim3(256), 0, s, P, L[0], L[1], L[2], dt,
                       hist_shift, parts, phist, Grid{}, 0.0, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL(k_reach_final, dim3(RHO_BINS / 256, REACH_FINAL_Y), dim3(256), 0, s, (int)g,
                     parts, phist, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a2: cell id + histogram

// Cell of each sphere and its rank within the cell (one atomic per sphere, or
// per run of spheres of one cell in consecutive lanes).
// Extent split: a sphere whose extent r + |v| dt exceeds rho_c goes to the
// second layer of cells (number G.layer2 + c), searched separately; the first
// layer then only needs cells of side 2 rho_c.  rho_c = +inf: one layer.
__global__ __launch_bounds__(256) void k_cell_hist(Particles P, Grid G, double dt, double rho_c,
                                                   int *cid, int *slot, int *count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int c = -1;
  if (i < P.n) {
    const int cx = cell_coord(P.x[i], G.inv_h[0], G.nc[0]);
    const int cy = cell_coord(P.y[i], G.inv_h[1], G.nc[1]);
    const int cz = cell_coord(P.z[i], G.inv_h[2], G.nc[2]);
    c = (cz * G.nc[1] + cy) * G.nc[0] + cx;
    if (G.layer2 && !(extent(P.r[i], P.vx[i], P.vy[i], P.vz[i], dt) <= rho_c)) c += G.layer2;
  }
  const int sl = run_slot(c, count);
  if (c >= 0) {
    cid[i] = c;
    slot[i] = sl;
  }
}

hipError_t launch_cell_hist(hipStream_t s, const Particles &P, const Grid &G, double dt,
                            double rho_c, int *cid, int *slot, int *count) {
  if (P.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_hist, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s, P, G, dt,
                     rho_c, cid, slot, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a3: exclusive scan

constexpr int SCAN_T = 1024;   // threads per scan block
constexpr int SCAN_E = 4;      // elements per thread
constexpr int SCAN_B = SCAN_T * SCAN_E;

// block-wide exclusive scan of one int per thread
__device__ void block_exclusive_scan(int v, int &excl) {
  __shared__ int wsum[SCAN_T / WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  int inc = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    int s = lane < SCAN_T / WAVE ? wsum[lane] : 0;
    int si = s;
    for (int o = 1; o < WAVE; o <<= 1) {
      const int t = __shfl_up(si, o);
      if (lane >= o) si += t;
    }
    if (lane < SCAN_T / WAVE) wsum[lane] = si - s;
  }
  __syncthreads();
  excl = wsum[w] + inc - v;
  __syncthreads();
}

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(const int *count, int n, int *start,
                                                         int *blocksum, ReachOut *out) {
  const int base = blockIdx.x * SCAN_B + threadIdx.x * SCAN_E;
  int v[SCAN_E];
  int sum = 0, mx = 0;
#pragma unroll
  for (int k = 0; k < SCAN_E; ++k) {
    v[k] = base + k < n ? count[base + k] : 0;
    sum += v[k];
    mx = v[k] > mx ? v[k] : mx;
  }
  int excl;
  block_exclusive_scan(sum, excl);
  int run = excl;
#pragma unroll
  for (int k = 0; k < SCAN_E; ++k) {
    if (base + k < n) start[base + k] = run;
    run += v[k];
  }
  // block total: the last thread's running end
  if (threadIdx.x == SCAN_T - 1) blocksum[blockIdx.x] = run;
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
  }
  __shared__ int wmax[SCAN_T / WAVE];
  if (__lane_id() == 0) wmax[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < SCAN_T / WAVE; ++k) mx = wmax[k] > mx ? wmax[k] : mx;
    atomicMax(&out->maxcell, (unsigned int)mx);
  }
}

// exclusive scan of the block sums in place (one block, chunks of SCAN_T)
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int *blocksum, int nb) {
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += SCAN_T) {
    const int i = c0 + threadIdx.x;
    const int v = i < nb ? blocksum[i] : 0;
    int excl;
    block_exclusive_scan(v, excl);
    const int c = carry;
    if (i < nb) blocksum[i] = c + excl;
    __syncthreads();
    if (threadIdx.x == SCAN_T - 1) carry = c + excl + v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int *start, const int *count, int n,
                                                  const int *blocksum) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int v = start[i] + blocksum[i / SCAN_B];
  start[i] = v;
  if (i == n - 1) start[n] = v + count[i];
}

hipError_t launch_scan(hipStream_t s, const int *count, int ncell, int *start, int *blocksum,
                       ReachOut *out) {
  const int nb = (ncell + SCAN_B - 1) / SCAN_B;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SCAN_T), 0, s, count, ncell, start, blocksum,
                     out);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, blocksum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((ncell + 255) / 256), dim3(256), 0, s, start, count, ncell,
                     blocksum);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a4: scatter

// cell-sorted 64-B records of the start-of-step state; reads the caller's SoA
// arrays coalesced and writes one record per sphere (its caller index and box
// inside, so no other array is written in sorted order).
__global__ __launch_bounds__(256) void k_scatter(Particles P, const int *cid, const int *slot,
                                                 const int *start, Rec *rec, int *rank,
                                                 const int *box_of, const unsigned int *flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= P.n || (flags && flags[FLAG_ERR])) return;
  const int c = cid[i];
  const int pos = start[c] + slot[i];
  Rec q;
  q.x = P.x[i];
  q.y = P.y[i];
  q.z = P.z[i];
  q.r = P.r[i];
  q.vx = P.vx[i];
  q.vy = P.vy[i];
  q.vz = P.vz[i];
  q.o = (int)i;
  q.box = box_of ? box_of[i] : 0;
  rec[pos] = q;
  rank[i] = pos;
}

hipError_t launch_scatter(hipStream_t s, const Particles &P, const int *cid, const int *slot,
                          const int *start, Rec *rec, int *rank, const BatchDev *B) {
  if (P.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s, P, cid,
                     slot, start, rec, rank, B ? B->box_of : nullptr,
                     B ? (const unsigned int *)B->flags : nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a5: sweep-1 detect

// All contacts within dt among all spheres (rule 1; eq. detect1/detect2), each
// unordered pair of spheres in neighbouring cells tested exactly once (the
// half stencil: own cell with j after i, and the 13 forward neighbour cells).
// Every contact (i, j, t) is appended to the contact slots of both spheres.
//
// One wave per home cell.  The wave's candidate list is the concatenation of
// up to 10 contiguous runs of the cell-sorted records (4 rows of 3 cells, the
// own cell and the next cell; a periodic wrap along x splits a row in two).
// Lanes hold candidates j (one 64-B record each, loaded once per chunk of 64);
// the home spheres i are wave-uniform and loop inside, so each pair costs the
// arithmetic only.  A run carries the periodic image shift of its cells; for a
// pair that can touch, the shifted separation equals the minimum image of rule
// 1 bitwise (the grid has >= 3 cells per axis and cell side >= reach).
//
// A conservative filter (pair64, pair32) keeps the square root, the division
// and the rule's exact operation order off the hot path; every pair it passes
// is decided by the rule itself.
constexpr int MAXRUN = 10;

// shift code of a run: per axis 0 = -L, 1 = none, 2 = +L (2 bits each), bit 6 = own cell
__device__ __forceinline__ int run_code(int sx, int sy, int sz, int own) {
  return (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4) | (own << 6);
}

// -L, 0 or +L for c = 0, 1, 2: (c - 1) L is each of them exactly (one convert
// and one multiply instead of a chain of selects).
__device__ __forceinline__ double code_shift(int c, double L) { return (double)(c - 1) * L; }

// One run of a home cell's candidate list in the wave's table in LDS: the
// offset from list slot to sorted index, the image code (run_code; bit 6 the
// own cell) and the image shift per axis, (c - 1) L (exact).
struct alignas(16) RunT {
  int off, code;
  double sx, sy, sz;
};

// Candidate slots past the end of the list hold this far-away sphere: its
// separation squares to +inf and b stays finite, so it never passes the reject.
constexpr double FAR_AWAY = 1e300;

// Append contact (i, j, t) to both spheres' slots.
__device__ __forceinline__ void record_contact(const DetectArgs &A, int i, int g, double t) {
  const int K = A.K;
  const size_t n = (size_t)A.n;
  const int k1 = atomicAdd(&A.cnt[i], 1);
  if (k1 < K) {
    A.slot_t[k1 * n + i] = t;
    A.slot_j[k1 * n + i] = g;
  }
  const int k2 = atomicAdd(&A.cnt[g], 1);
  if (k2 < K) {
    A.slot_t[k2 * n + g] = t;
    A.slot_j[k2 * n + g] = i;
  }
}


// Filter survivors of one wave awaiting the exact rule: (home i, candidate g)
// pairs in the wave's LDS queue.  A survivor is rare (about one per home
// sphere); deciding it at once would run the square root, the division and
// two atomics for one live lane while the other 63 idle, so survivors are
// queued and decided 64 at a time at the end of the home cell, where few
// registers are live.  A survivor that finds the queue full is decided at
// once.
constexpr int QCAP = 256;

struct SurvivorQueue {
  int2 *q;              // cap entries in LDS, private to the wave
  int n;                // entries waiting (wave-uniform)
  unsigned int pushed;  // survivors seen (wave-uniform)
  int cap;
  unsigned long long tests;  // unordered pairs tested (wave-uniform)
};

// The rule for every queued pair (rule 1 with the canonical minimum image,
// which for every pair that can touch is the image the stencil tested, and
// for any other pair finds no contact either).
__device__ __forceinline__ void flush_survivors(const DetectArgs &A, const Grid &G,
                                                SurvivorQueue &Q) {
  for (int e0 = 0; e0 < Q.n; e0 += WAVE) {
    const int e = e0 + (int)__lane_id();
    if (e < Q.n) {
      const int2 pr = Q.q[e];
      const Rec a = A.rec[pr.x], b = A.rec[pr.y];
      double t;
      if (pair_time(a, b, G, A.dt, t)) record_contact(A, pr.x, pr.y, t);
    }
  }
  Q.n = 0;
}

// Queue this lane's survivor (i, g) if `pass`; returns false if the queue had
// no room for the wave's survivors, which the caller then decides at once.
__device__ __forceinline__ bool push_survivor(bool pass, int i, int g, SurvivorQueue &Q) {
  const unsigned long long m = __ballot(pass);
  if (!m) return true;
  const int c = __popcll(m);
  Q.pushed += c;
  if (Q.n + c > Q.cap) return false;
  if (pass) {
    const unsigned int lane = __lane_id();
    Q.q[Q.n + __popcll(m & ((1ull << lane) - 1ull))] = make_int2(i, g);
  }
  Q.n += c;
  return true;
}

// Append the survivors of two home spheres i0 and i1 against the lane's
// candidate g (pass flags p0 and p1) to the queue, which has room for two
// wave's worth (the caller makes sure of it).  One wave-wide test when neither
// passes anywhere, the common case.
__device__ __forceinline__ void push_two(bool p0, bool p1, int i0, int i1, int g,
                                         SurvivorQueue &Q) {
  const unsigned long long m0 = __ballot(p0), m1 = __ballot(p1);
  if (!(m0 | m1)) return;
  const unsigned long long below = (1ull << __lane_id()) - 1ull;
  const int c0 = __popcll(m0), c1 = __popcll(m1);
  if (p0) Q.q[Q.n + __popcll(m0 & below)] = make_int2(i0, g);
  if (p1) Q.q[Q.n + c0 + __popcll(m1 & below)] = make_int2(i1, g);
  Q.n += c0 + c1;
  Q.pushed += c0 + c1;
}

// One home sphere (FP32 record) against the lane's candidate: the same filter in
// binary32 with the contact distance inflated by the band.  Survivors are
// decided by the binary64 rule (flush_survivors).
template <bool MASK>
__device__ __forceinline__ bool pass32(const DetectArgs &A, int thr, float bx, float by, float bz,
                                       float br, float bvx, float bvy, float bvz, int i,
                                       const Rec32 &h) {
  const float d0 = bx - h.x, d1 = by - h.y, d2 = bz - h.z;
  const float u0 = bvx - h.vx, u1 = bvy - h.vy, u2 = bvz - h.vz;
  const float sb = (h.r + br) * A.kband;
  const float bb = __builtin_fmaf(d0, u0, __builtin_fmaf(d1, u1, d2 * u2));
  const float q = __builtin_fmaf(d0, d0, __builtin_fmaf(d1, d1, d2 * d2));
  const float cc = __builtin_fmaf(-sb, sb, q);
  return (!MASK || i < thr) && __builtin_fmaf(bb, A.dt2f, cc) <= 0.0f;
}

// One candidate chunk against the homes [h0, h1) staged in LDS at p.
template <bool MASK>
__device__ __forceinline__ void detect_chunk32(const DetectArgs &A, const Grid &G, const Rec32 *p, int h0,
                                               int h1, int g, int thr, const RunT &run, double ox,
                                               double oy, double oz, SurvivorQueue &Q) {
  float bx, by, bz, bvx, bvy, bvz, br;
  if (thr >= 0) {
    const Rec b = A.rec[g];
    // candidate relative to the home cell centre (ox, oy, oz), image shift applied
    bx = (float)((b.x + run.sx) - ox);
    by = (float)((b.y + run.sy) - oy);
    bz = (float)((b.z + run.sz) - oz);
    bvx = (float)b.vx;
    bvy = (float)b.vy;
    bvz = (float)b.vz;
    br = (float)b.r;
  } else {
    bx = by = bz = 1e18f;
    bvx = bvy = bvz = 0.f;
    br = 0.f;
  }
  int i = h0;
  for (;;) {
    // two homes per step while the queue has room for their survivors; a full
    // queue (rare) is decided here, outside the loop
    for (; i < h1 && Q.n <= Q.cap - 2 * WAVE; i += 2) {
      const bool two = i + 1 < h1;  // an odd last home pairs with itself, never passing twice
      const Rec32 ha = p[i - h0], hb = p[two ? i + 1 - h0 : i - h0];
      const bool p0 = pass32<MASK>(A, thr, bx, by, bz, br, bvx, bvy, bvz, i, ha);
      const bool p1 = two && pass32<MASK>(A, thr, bx, by, bz, br, bvx, bvy, bvz, i + 1, hb);
      push_two(p0, p1, i, i + 1, g, Q);
    }
    if (i >= h1) break;
    flush_survivors(A, G, Q);
  }
}

// Pair tests of one home cell (see k_detect_half).  `start` points at the first
// cell of the box whose grid is G (cell numbers below are local to that box;
// sphere positions in start[] are global).
// Runs of consecutive cell-sorted records that make the half stencil of one
// home cell: run 0 the own cell (pairs with j after i), run 1 the next cell
// along x, runs 2..9 the 4 rows of 3 cells, each row as two runs (the second
// empty unless the row wraps along x); each with its periodic image code.
// Run k's bounds are the starts of two cells, held in lanes 2k and 2k + 1 of
// the wave, so that one vector load fetches all 20 and the runs are formed
// lane by lane rather than in scalar code.

// Lane j < 20 of a home cell's stencil: the cell whose start it loads (lane
// 2k the first cell of run k, lane 2k + 1 the cell one past its last) and run
// k's image code (run_code).  Lanes from 20 on load nothing.
__device__ __forceinline__ int cell_starts(const Grid &G, const int *start, int cell, int &code) {
  const int nc0 = G.nc[0], nc1 = G.nc[1], nc2 = G.nc[2];
  int cx, cy, cz;
  cell_xyz(G, cell, cx, cy, cz);
  // the lane index made opaque per call, so that the lane-constant selections
  // below are recomputed per cell rather than hoisted out of a cell loop
  // (held across it they cost registers and, in the grouped kernel, spills)
  int ln = (int)__lane_id();
  asm volatile("" : "+v"(ln));
  const int k = ln >> 1, end = ln & 1;
  const bool lw = cx - 1 < 0, rw = cx + 1 >= nc0;  // the row wraps left / right
  // rows (runs 2..9): offsets (dy, dz) = (1, 0), (-1, 1), (0, 1), (1, 1)
  const int row = (k - 2) >> 1, second = (k - 2) & 1;
  int y = cy + (row == 1 ? -1 : (row == 2 ? 0 : 1)), z = cz + (row == 0 ? 0 : 1);
  const int sy = y >= nc1 ? 1 : (y < 0 ? -1 : 0), sz = z >= nc2 ? 1 : 0;
  y -= sy * nc1;
  z -= sz * nc2;
  // a row's two runs, as cells [a0, a1) and [a2, a3) of the row: the wrapped
  // left cell then cells 0..1; cells cx-1..cx then the wrapped right cell 0;
  // or cells cx-1..cx+1 and an empty second run.  The four bounds are uniform
  // and each lane selects one (simple selects, no divergent branches).
  const int a0 = lw ? nc0 - 1 : cx - 1, a1 = lw ? nc0 : (rw ? cx + 1 : cx + 2);
  const int a2 = lw || rw ? 0 : cx + 2, a3 = lw ? 2 : (rw ? 1 : cx + 2);
  const int o01 = end ? a1 : a0, o23 = end ? a3 : a2;
  const int o = second ? o23 : o01;
  // image along x of a row's first / second run
  const int sx0 = lw ? -1 : 0, sx1 = !lw && rw ? 1 : 0;
  const int sx_row = second ? sx1 : sx0;
  // run 1: the next cell along x, cell 0 of the own row where x wraps
  const int c01 = k == 0 ? cell : (rw ? cell - cx : cell + 1);
  const int idx = k < 2 ? c01 + end : (z * nc1 + y) * nc0 + o;
  const int code01 = k == 0 ? run_code(0, 0, 0, 1) : run_code(rw ? 1 : 0, 0, 0, 0);
  code = k < 2 ? code01 : run_code(sx_row, sy, sz, 0);
  int v = 0;
  if (ln < 20) v = start[idx];
  return v;
}

// A home cell's runs as the candidate search needs them: its spheres [h0, h1),
// the candidate list length, and the first list slot of each run (pre[0] = 0;
// an empty run starts where the next does).
struct CellSet {
  int h0, h1, total;
  int pre[MAXRUN];
};

// The runs of a home cell from its lanes' starts v and codes (cell_starts):
// run lengths and their prefix sums formed across lanes 0..19 (DPP shifts
// within rows of 16 lanes, then the carry of the first row), and the run table
// rt (the wave's own room in LDS; its LDS operations stay in order) written by
// lanes 2k: run k's offset from list slot to sorted index, its code and its
// image shift on the grid G.  Returns false for an empty home cell.
__device__ __forceinline__ bool cell_setup(const Grid &G, int v, int code, RunT *rt, CellSet &S) {
  const int h0 = __builtin_amdgcn_readlane(v, 0), h1 = __builtin_amdgcn_readlane(v, 1);
  S.h0 = h0;
  S.h1 = h1;
  if (h1 <= h0) return false;
  // the lane index opaque, so that the table addresses are formed here per
  // cell and not held across the cell loop (registers)
  int ln = (int)__lane_id();
  asm volatile("" : "+v"(ln));
  const bool first = ln < 20 && (ln & 1) == 0;
  // lane 2k + 1's start beside lane 2k's (row_shl:1; a pair never straddles a row)
  const int vn = __builtin_amdgcn_update_dpp(0, v, 0x101, 0xf, 0xf, true);
  const int rl = first ? vn - v : 0;
  int inc = rl;
  inc += __builtin_amdgcn_update_dpp(0, inc, 0x111, 0xf, 0xf, true);  // row_shr:1
  inc += __builtin_amdgcn_update_dpp(0, inc, 0x112, 0xf, 0xf, true);  // row_shr:2
  inc += __builtin_amdgcn_update_dpp(0, inc, 0x114, 0xf, 0xf, true);  // row_shr:4
  inc += __builtin_amdgcn_update_dpp(0, inc, 0x118, 0xf, 0xf, true);  // row_shr:8
  const int carry = __builtin_amdgcn_readlane(inc, 15);
  if (ln >= 16) inc += carry;
  const int excl = inc - rl;
  if (first)
    rt[ln >> 1] = RunT{v - excl, code, code_shift(code & 3, G.sL[0]),
                       code_shift((code >> 2) & 3, G.sL[1]), code_shift((code >> 4) & 3, G.sL[2])};
  S.total = __builtin_amdgcn_readlane(inc, 19);
  S.pre[0] = 0;
#pragma unroll
  for (int k = 1; k < MAXRUN; ++k) S.pre[k] = __builtin_amdgcn_readlane(excl, 2 * k);
  return true;
}


// Home spheres of the binary32 filter staged in LDS per batch.
constexpr int HB32 = WAVE;

// Pair tests of one home cell with the binary32 filter.  The home spheres are
// staged in LDS (hl) HB32 at a time as binary32 records relative to the home
// cell centre, converted from the binary64 records; candidates in chunks of 64
// lanes, converted likewise with their run's image shift.  rt: the wave's room
// in LDS for the cell's run table (MAXRUN entries).
__device__ __forceinline__ void detect_cell32(const DetectArgs &A, const Grid &G, const int *start,
                                              int cell, SurvivorQueue &Q, Rec32 *hl, RunT *rt) {
  int code;
  const int vs = cell_starts(G, start, cell, code);
  CellSet S;
  if (!cell_setup(G, vs, code, rt, S)) return;
  const int h0 = S.h0, h1 = S.h1, total = S.total;
  const int *pre = S.pre;
  const int lane = __lane_id();
  // unordered pairs this cell tests: own cell pairs once, every home against the rest
  Q.tests += (unsigned long long)(h1 - h0) * (unsigned long long)(total - (h1 - h0)) +
             (unsigned long long)(h1 - h0) * (unsigned long long)(h1 - h0 - 1) / 2ull;
  int cx, cy, cz;
  cell_xyz(G, cell, cx, cy, cz);
  const double ox = (cx + 0.5) * G.h[0], oy = (cy + 0.5) * G.h[1], oz = (cz + 0.5) * G.h[2];
  for (int hb = h0; hb < h1; hb += HB32) {
    const int he = hb + HB32 < h1 ? hb + HB32 : h1;
    if (hb + lane < he) {
      const Rec q = A.rec[hb + lane];
      Rec32 f;
      f.x = (float)(q.x - ox);
      f.y = (float)(q.y - oy);
      f.z = (float)(q.z - oz);
      f.r = (float)q.r;
      f.vx = (float)q.vx;
      f.vy = (float)q.vy;
      f.vz = (float)q.vz;
      f.pad = 0.f;
      hl[lane] = f;
    }
    __syncthreads();  // the workgroup is this one wave
    for (int base = 0; base < total; base += WAVE) {
      const int v = base + lane;
      int r = 0;  // the run of list slot v (see detect_cell64)
#pragma unroll
      for (int k = 1; k < MAXRUN; ++k) r += v >= pre[k] ? 1 : 0;
      asm volatile("" : "+v"(r));  // the count apart from the table address
      const RunT run = rt[r];
      const int g = run.off + v;
      const bool ok = v < total;
      const bool own = (run.code >> 6) & 1;
      const int thr = !ok ? -1 : (own ? g : 0x7fffffff);
      if (base < h1 - h0)
        detect_chunk32<true>(A, G, (const Rec32 *)hl, hb, he, g, thr, run, ox, oy, oz, Q);
      else
        detect_chunk32<false>(A, G, (const Rec32 *)hl, hb, he, g, thr, run, ox, oy, oz, Q);
    }
    __syncthreads();  // before the next batch overwrites hl
  }
  // the survivors left in Q are the caller's to decide
}

// ---------------------------------------------------------------- a5, binary64 Gram filter

// The binary64 filter in Gram form.  With positions relative to the home cell
// centre o, F = |d|^2 - s^2 + dt2 (d . u) = alpha_i + beta_j + <P_j, Q_i> where
//   P_j = (x_j, v_j, r_j),  Q_i = (-2 x_i - dt2 v_i, -dt2 x_i, -2 r_i),
//   alpha_i = |x_i|^2 + dt2 x_i.v_i - r_i^2,  beta_j = |x_j|^2 + dt2 x_j.v_j - r_j^2
// (d = x_j - x_i, u = v_j - v_i, s = r_i + r_j).  Q_i and alpha_i are formed once
// per home sphere into LDS, P_j and the candidate's threshold tol64 - beta_j
// once per candidate and chunk (the run's periodic shift applied), so a pair
// costs seven FMAs (alpha_i + <P_j, Q_i>, alpha_i the first addend) and one
// compare.  A pair passes iff alpha_i + <P_j, Q_i> <= tol64 - beta_j as
// evaluated, tol64 a bound on the rounding of this evaluation, of the
// threshold and of the relative coordinates for pairs the rule can keep (host,
// gram64_tolerance); survivors are decided by the rule (flush_survivors), so
// the result is exactly the rule's.
struct alignas(16) HomeQ {
  double q[7];
  double alpha;
};

// Pair tests of one candidate chunk against a batch of homes, two homes per
// step; a survivor that finds the queue full is decided at once.
template <bool MASK>
__device__ __forceinline__ void detect_chunk64(const DetectArgs &A, const Grid &G, const HomeQ *hq,
                                               int nb, int i0, int g, int thr, const double P[7],
                                               double fthr, SurvivorQueue &Q) {
  int k = 0;
  for (; k + 1 < nb; k += 2) {
    const HomeQ a = hq[k], b = hq[k + 1];
    double t0 = a.alpha, t1 = b.alpha;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      t0 = __builtin_fma(P[c], a.q[c], t0);
      t1 = __builtin_fma(P[c], b.q[c], t1);
    }
    const int i = i0 + k;
    const bool p0 = t0 <= fthr && (!MASK || i < thr);
    const bool p1 = t1 <= fthr && (!MASK || i + 1 < thr);
    if (!push_survivor(p0, i, g, Q) && p0) {
      double t;
      if (pair_time(A.rec[i], A.rec[g], G, A.dt, t)) record_contact(A, i, g, t);
    }
    if (!push_survivor(p1, i + 1, g, Q) && p1) {
      double t;
      if (pair_time(A.rec[i + 1], A.rec[g], G, A.dt, t)) record_contact(A, i + 1, g, t);
    }
  }
  if (k < nb) {
    const HomeQ a = hq[k];
    double t0 = a.alpha;
#pragma unroll
    for (int c = 0; c < 7; ++c) t0 = __builtin_fma(P[c], a.q[c], t0);
    const int i = i0 + k;
    const bool p0 = t0 <= fthr && (!MASK || i < thr);
    if (!push_survivor(p0, i, g, Q) && p0) {
      double t;
      if (pair_time(A.rec[i], A.rec[g], G, A.dt, t)) record_contact(A, i, g, t);
    }
  }
}

// Pair tests of one home cell with the binary64 Gram filter; homes in batches
// of 64 (hq holds one batch), candidates in chunks of 64 lanes.
// vs, code: the cell's 20 starts and run codes (cell_starts), loaded ahead by
// the caller; rt: the wave's room in LDS for the cell's run table (MAXRUN
// entries).
__device__ __forceinline__ void detect_cell64(const DetectArgs &A, const Grid &G, int vs,
                                              int code, int cell, SurvivorQueue &Q, HomeQ *hq,
                                              RunT *rt) {
  CellSet S;
  if (!cell_setup(G, vs, code, rt, S)) return;
  const int h0 = S.h0, h1 = S.h1, nh = h1 - h0, total = S.total;
  const int *pre = S.pre;
  Q.tests += (unsigned long long)nh * (unsigned long long)(total - nh) +
             (unsigned long long)nh * (unsigned long long)(nh - 1) / 2ull;
  const int lane = __lane_id();
  int cx, cy, cz;
  cell_xyz(G, cell, cx, cy, cz);
  const double ox = (cx + 0.5) * G.h[0], oy = (cy + 0.5) * G.h[1], oz = (cz + 0.5) * G.h[2];
  const double dt2 = A.dt2;
  for (int hb = 0; hb < nh; hb += WAVE) {
    const int nb = nh - hb < WAVE ? nh - hb : WAVE;
    if (lane < nb) {  // this batch's home terms (one wave owns hq: in-order LDS)
      const Rec a = A.rec[h0 + hb + lane];
      const double xh = a.x - ox, yh = a.y - oy, zh = a.z - oz;
      HomeQ h;
      h.q[0] = -2.0 * xh - dt2 * a.vx;
      h.q[1] = -2.0 * yh - dt2 * a.vy;
      h.q[2] = -2.0 * zh - dt2 * a.vz;
      h.q[3] = -dt2 * xh;
      h.q[4] = -dt2 * yh;
      h.q[5] = -dt2 * zh;
      h.q[6] = -2.0 * a.r;
      h.alpha = ((xh * xh + yh * yh) + zh * zh) + dt2 * ((xh * a.vx + yh * a.vy) + zh * a.vz) -
                a.r * a.r;
      hq[lane] = h;
    }
    for (int base = 0; base < total; base += WAVE) {
      const int v = base + lane;
      // the run of list slot v: the last run whose first slot is at most v.  The
      // first slots are non-decreasing, so it is the number of runs after the
      // first that start at or before v (an empty run starts where the next
      // does, so it is never the one counted last for a slot inside the list)
      int r = 0;
#pragma unroll
      for (int k = 1; k < MAXRUN; ++k) r += v >= pre[k] ? 1 : 0;
      asm volatile("" : "+v"(r));  // the count apart from the table address
      const RunT run = rt[r];
      const int g = run.off + v;
      const bool ok = v < total;
      const bool own = (run.code >> 6) & 1;
      const int thr = !ok ? -1 : (own ? g : 0x7fffffff);
      double P[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      double beta = 1e300;  // no candidate: its threshold -1e300 is never met
      if (thr >= 0) {
        const Rec b = A.rec[g];
        const double xj = (b.x + run.sx) - ox;
        const double yj = (b.y + run.sy) - oy;
        const double zj = (b.z + run.sz) - oz;
        P[0] = xj;
        P[1] = yj;
        P[2] = zj;
        P[3] = b.vx;
        P[4] = b.vy;
        P[5] = b.vz;
        P[6] = b.r;
        beta = ((xj * xj + yj * yj) + zj * zj) + dt2 * ((xj * b.vx + yj * b.vy) + zj * b.vz) -
               b.r * b.r;
      }
      // own-cell candidates (the first rl[0] of the list): only j after i
      if (base < nh)
        detect_chunk64<true>(A, G, hq, nb, h0 + hb, g, thr, P, A.tol64 - beta, Q);
      else
        detect_chunk64<false>(A, G, hq, nb, h0 + hb, g, thr, P, A.tol64 - beta, Q);
    }
  }
  // the survivors left in Q are the caller's to decide (flush_survivors), now
  // or after later cells of the same grid
}

template <bool FP32>
__global__ __launch_bounds__(WAVE) void k_detect_half(DetectArgs A) {
  __shared__ int2 survq[QCAP];
  SurvivorQueue Q{survq, 0, 0u, QCAP, 0ull};
  if (FP32) {  // A.cpw consecutive cells per workgroup (see k_detect_half64g)
    __shared__ Rec32 hl[HB32];
    __shared__ RunT rt[MAXRUN];
    const int c0 = xcd_remap(blockIdx.x, gridDim.x) * A.cpw;
    const int c1 = c0 + A.cpw < A.G.ncell ? c0 + A.cpw : A.G.ncell;
    for (int cell = c0; cell < c1; ++cell) {
      detect_cell32(A, A.G, A.start, cell, Q, hl, rt);
      if (cell + 1 == c1 || Q.n >= WAVE) flush_survivors(A, A.G, Q);
    }
  } else {
    __shared__ HomeQ hq[WAVE];
    __shared__ RunT rt[MAXRUN];
    const int cell = xcd_remap(blockIdx.x, gridDim.x);
    int code;
    const int vs = cell_starts(A.G, A.start, cell, code);
    detect_cell64(A, A.G, vs, code, cell, Q, hq, rt);
    flush_survivors(A, A.G, Q);
  }
  // this cell's counts, summed by launch_cell_counts (a counter atomic per
  // wave would serialise over the million cells)
  if (__lane_id() == 0) A.cellc[blockIdx.x] = CellCount{Q.tests, FP32 ? Q.pushed : 0ull};
}

// The binary64 filter over A.cpw consecutive cells per workgroup, for sparse
// cells: the survivor queue carries over between them and is decided a wave at
// a time (a cell of 13 spheres leaves about 13 survivors, so deciding them
// per cell runs the rule's square root and division on a fifth of the lanes).
// Register-limited to 5 waves per SIMD (96 registers, no spills).
__global__ __launch_bounds__(WAVE, 5) void k_detect_half64g(DetectArgs A) {
  __shared__ int2 survq[QCAP];
  __shared__ HomeQ hq[WAVE];
  __shared__ RunT rt[MAXRUN];
  SurvivorQueue Q{survq, 0, 0u, QCAP, 0ull};
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * A.cpw;
  const int c1 = c0 + A.cpw < A.G.ncell ? c0 + A.cpw : A.G.ncell;
  // the next cell's starts are loaded while this cell is tested
  int code = 0;
  int v = c0 < c1 ? cell_starts(A.G, A.start, c0, code) : 0;
  for (int cell = c0; cell < c1; ++cell) {  // one flush site (register pressure)
    const int vc = v;
    const int cc = code;
    if (cell + 1 < c1) v = cell_starts(A.G, A.start, cell + 1, code);
    detect_cell64(A, A.G, vc, cc, cell, Q, hq, rt);
    if (cell + 1 == c1 || Q.n >= WAVE) flush_survivors(A, A.G, Q);
  }
  if (__lane_id() == 0) A.cellc[blockIdx.x] = CellCount{Q.tests, 0ull};
}

// Workgroups of launch_detect_half (one wave each): one per cell, but for the
// persistent binary64 kernel a multiple of 8 (the XCDs) near the waves the
// chip holds at once.  Also the number of per-workgroup counts it writes.
int detect_half_blocks(const DetectArgs &A) {
  if (A.cpw <= 1) return A.G.ncell;
  return (A.G.ncell + A.cpw - 1) / A.cpw;
}

// Box of a global cell number: the last b with cell_base[b] <= c.
__device__ __forceinline__ int box_of_cell(const int *cell_base, int nbox, int c) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell_base[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Batched form: the cells of all boxes are numbered consecutively, box after
// box, and each workgroup (one wave) takes cpw consecutive global cells, as
// k_detect_half64g does in one box: the box of each cell comes from the
// first-cell table, the pair tests run with that box's grid, and the survivor
// queue carries over the cells, decided with the grid of the box its survivors
// came from whenever the next cell lies in another box, when it holds a wave's
// worth, and at the end.
__global__ __launch_bounds__(WAVE) void k_detect_batched(DetectArgs A, BatchDev B, int cpw) {
  if (B.flags[FLAG_ERR]) return;
  __shared__ int2 survq[QCAP];
  __shared__ HomeQ hq[WAVE];
  __shared__ RunT rt[MAXRUN];
  SurvivorQueue Q{survq, 0, 0u, QCAP, 0ull};
  const int total = B.cell_base[B.nbox];
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * cpw;
  const int c1 = c0 + cpw < total ? c0 + cpw : total;
  if (c0 >= c1) return;
  int b = box_of_cell(B.cell_base, B.nbox, c0);
  int qb = b;  // the box of the queued survivors
  for (int item = c0; item < c1; ++item) {
    while (item >= B.cell_base[b + 1]) ++b;  // boxes of no cells are passed over
    if (b != qb) {
      if (Q.n > 0) flush_survivors(A, B.gtab[qb], Q);
      qb = b;
    }
    const Grid G = B.gtab[b];
    const int base = B.cell_base[b];
    int code;
    const int vs = cell_starts(G, A.start + base, item - base, code);
    detect_cell64(A, G, vs, code, item - base, Q, hq, rt);
    if (item + 1 == c1 || Q.n >= WAVE) flush_survivors(A, G, Q);
  }
}

// Sum of the per-cell counts of the k_detect_half kernels (a few cells per
// thread, so the loads of a thread are few and in flight together; one atomic
// per workgroup and counter, spread over the shards).
__global__ __launch_bounds__(256) void k_cell_counts(const CellCount *c, int n,
                                                     SweepCounters *ctr) {
  unsigned long long t = 0ull, r = 0ull;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    t += c[i].tests;
    r += c[i].recheck;
  }
  block_add(t, &my_shard(ctr).tests);
  block_add(r, &my_shard(ctr).recheck);
}

hipError_t launch_cell_counts(hipStream_t s, const CellCount *c, int n, SweepCounters *ctr) {
  if (n <= 0) return hipSuccess;
  int g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_cell_counts, dim3(g), dim3(256), 0, s, c, n, ctr);
  return hipGetLastError();
}

hipError_t launch_detect_half(hipStream_t s, const DetectArgs &A) {
  if (A.G.ncell <= 0) return hipSuccess;
  if (A.fp32)
    hipLaunchKernelGGL(k_detect_half<true>, dim3(detect_half_blocks(A)), dim3(WAVE), 0, s, A);
  else if (A.cpw > 1)
    hipLaunchKernelGGL(k_detect_half64g, dim3(detect_half_blocks(A)), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL(k_detect_half<false>, dim3(A.G.ncell), dim3(WAVE), 0, s, A);
  return hipGetLastError();
}


// ---------------------------------------------------------------- a5/a7: partner from contact slots

// Earliest partner (rule 2: exact binary64 t, ties to the smaller caller index)
// of each sphere among its recorded contacts whose partner has not collided;
// with crank given (the literal order), the contact of smallest curve rank
// instead (see k_curve_rank).  The contact set of a sphere only shrinks over
// the sweeps of a step, so the slots written by the sweep-1 detect are
// complete for every later sweep.
// first = 1: every sphere (sweep 1); first = 0: only DIRTY spheres, which
// become ACTIVE again.  Spheres with more contacts than slots are queued for
// the exact search (rare; one atomic per wave that has one).  Slots are
// k-major, so the reads of a wave are coalesced.
__global__ __launch_bounds__(256) void k_slot_min(int n, int first, const int *cnt,
                                                  const double *slot_t, const int *slot_j, int K,
                                                  uint8_t *status, const Rec *rec, int *key_j,
                                                  double *key_t, int *ovf_list,
                                                  SweepCounters *ctr, const unsigned int *flags,
                                                  const int *list, int nlist, Grid G,
                                                  const unsigned long long *crank) {
  if (flags && (flags[FLAG_ERR] || flags[FLAG_DONE])) return;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int i = list && t < nlist ? list[t] : t;
  bool ovf = false;
  unsigned long long nc = 0ull;
  if (list ? t < nlist : i < n) {
    const uint8_t st = status[i];
    if (first ? st == ST_ACTIVE : st == ST_DIRTY) {
      const int c = cnt[i];
      nc = (unsigned long long)c;
      if (c > K) {
        ovf = true;
        key_j[i] = -1;
        key_t[i] = INFINITY;
      } else {
        double bt = INFINITY;
        int bj = -1;
        unsigned long long br = ~0ull;  // literal order: curve rank of the best contact
        // between walls a contact counts only before both centres reach a wall
        double ti = INFINITY;
        if (G.walls) {
          const Rec a = rec[i];
          ti = time_to_wall(a.x, a.y, a.z, a.vx, a.vy, a.vz, G);
        }
        for (int k = 0; k < c; ++k) {
          const int j = slot_j[(size_t)k * n + i];
          if (!first && status[j] == ST_COLLIDED) continue;
          const double t = slot_t[(size_t)k * n + i];
          if (G.walls) {
            const Rec b = rec[j];
            if (!(t <= ti) || !(t <= time_to_wall(b.x, b.y, b.z, b.vx, b.vy, b.vz, G))) continue;
          }
          if (crank) {
            const unsigned long long rj = crank[j];
            if (rj < br) {
              br = rj;
              bt = t;
              bj = j;
            }
          } else if (t < bt || (bj >= 0 && t == bt && rec[j].o < rec[bj].o)) {
            bt = t;
            bj = j;
          }
        }
        key_j[i] = bj;
        key_t[i] = bt;
      }
      if (!first) status[i] = ST_ACTIVE;
    }
  }
  const unsigned int k = wave_append(ovf, &ctr->n_overflow);
  if (ovf) ovf_list[k] = i;
  if (first) block_add(nc, &my_shard(ctr).contacts);
}

hipError_t launch_slot_min(hipStream_t s, int n, int first, const int *cnt, const double *slot_t,
                           const int *slot_j, int K, uint8_t *status, const Rec *rec, int *key_j,
                           double *key_t, int *ovf_list, SweepCounters *ctr,
                           const unsigned int *flags, const int *list, int nlist,
                           const Grid *G, const unsigned long long *crank) {
  const int items = list ? nlist : n;
  if (items <= 0) return hipSuccess;
  const Grid none{};  // walls = 0: periodic
  hipLaunchKernelGGL(k_slot_min, dim3((items + 255) / 256), dim3(256), 0, s, n, first, cnt, slot_t,
                     slot_j, K, status, rec, key_j, key_t, ovf_list, ctr, flags, list, nlist,
                     G ? *G : none, crank);
  return hipGetLastError();
}

// ---------------------------------------------------------------- the literal order's ranks

// Morton (Z-order) code of a cell: the bits of cx, cy, cz (each below 2^11)
// interleaved, x lowest.
__device__ __forceinline__ unsigned long long morton3(unsigned int cx, unsigned int cy,
                                                      unsigned int cz) {
  unsigned long long k = 0ull;
#pragma unroll
  for (int b = 0; b < 11; ++b) {
    k |= (unsigned long long)((cx >> b) & 1u) << (3 * b);
    k |= (unsigned long long)((cy >> b) & 1u) << (3 * b + 1);
    k |= (unsigned long long)((cz >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

// Rank of every sphere in the order the paper's traversal visits it (Sec.
// "Collision Operator": elements along a space-filling curve, particles of an
// element one after another): the Morton code of its cell on the curve grid C
// (nc cells of side h per axis) above its caller index,
// crank = code << 31 | o, in cell-sorted order.  A sphere's cell is
// floor(x / h) in binary64, clamped to nc - 1.
__global__ __launch_bounds__(256) void k_curve_rank(const Rec *rec, int n, CurveGrid C,
                                                    unsigned long long *crank) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const Rec a = rec[i];
  const double p[3] = {a.x, a.y, a.z};
  unsigned int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double q = floor(p[k] / C.h[k]);
    if (q < 0.0) q = 0.0;
    if (q > (double)(C.nc[k] - 1)) q = (double)(C.nc[k] - 1);
    c[k] = (unsigned int)q;
  }
  crank[i] = morton3(c[0], c[1], c[2]) << 31 | (unsigned long long)(unsigned int)a.o;
}

hipError_t launch_curve_rank(hipStream_t s, const Rec *rec, int n, const CurveGrid &C,
                             unsigned long long *crank) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_curve_rank, dim3((n + 255) / 256), dim3(256), 0, s, rec, n, C, crank);
  return hipGetLastError();
}

// ---------------------------------------------------------------- exact neighbourhood search

// Search box of a sphere in cell (cx, cy, cz): kx..kz cells either side along
// each axis, or the whole axis once when 2k + 1 covers it.  Calls
// run(first, end) for each run of consecutive sorted records (a row of cells
// along x, split in two where it wraps) of the layer whose first cell is
// `base`.  Every cell of the box is visited exactly once.
template <typename F>
__device__ __forceinline__ void search_box_runs(const Grid &G, const int *start, int base, int cx,
                                                int cy, int cz, const int k[3], F run) {
  const int nc0 = G.nc[0], nc1 = G.nc[1], nc2 = G.nc[2];
  const bool fx = 2 * k[0] + 1 >= nc0, fy = 2 * k[1] + 1 >= nc1, fz = 2 * k[2] + 1 >= nc2;
  const int ny = fy ? nc1 : 2 * k[1] + 1, nz = fz ? nc2 : 2 * k[2] + 1;
  for (int iz = 0; iz < nz; ++iz) {
    const int z = fz ? iz : (cz - k[2] + iz + nc2) % nc2;
    for (int iy = 0; iy < ny; ++iy) {
      const int y = fy ? iy : (cy - k[1] + iy + nc1) % nc1;
      const int row = base + (z * nc1 + y) * nc0;
      if (fx) {
        run(start[row], start[row + nc0]);
      } else {
        const int x0 = cx - k[0], x1 = cx + k[0];
        if (x0 < 0) {
          run(start[row + x0 + nc0], start[row + nc0]);
          run(start[row], start[row + x1 + 1]);
        } else if (x1 >= nc0) {
          run(start[row + x0], start[row + nc0]);
          run(start[row], start[row + x1 - nc0 + 1]);
        } else {
          run(start[row + x0], start[row + x1 + 1]);
        }
      }
    }
  }
}

// Cells either side of sphere a that can hold a partner: 1 when the cell side
// is at least the reach (one layer), else enough to cover the sphere's extent
// plus the largest extent (split grid).
__device__ __forceinline__ void search_radius(const Grid &G, const Rec &a, double dt, int k[3]) {
  if (G.rho_max > 0.0) {
    const double R = (extent(a.r, a.vx, a.vy, a.vz, dt) + G.rho_max) * (1.0 + 1e-9);
    for (int ax = 0; ax < 3; ++ax) k[ax] = (int)ceil(R / G.h[ax]);
  } else {
    k[0] = k[1] = k[2] = 1;
  }
}

// Distance along one axis from a sphere at offset f within its cell (cell side
// h) to the cells `o` cells away: 0 for its own cell, else the gap to the
// nearer face.  Cell faces are taken `eta` nearer, which covers spheres that
// rounding placed in a neighbouring cell.
__device__ __forceinline__ double face_gap(int o, double f, double h, double eta) {
  double g = 0.0;
  if (o > 0) g = o * h - f;
  if (o < 0) g = f - (o + 1) * h;
  g -= eta;
  return g > 0.0 ? g : 0.0;
}

// Run r of the ball-pruned search of a sphere at (px, py, pz) in cell
// (cx, cy, cz): r = (layer * nz + iz) * ny + iy) * 2 + part over the rows of
// its search box (kx..kz cells either side, whole axes once when 2k + 1 covers
// them).  A row is clipped along x to the cells within distance R[layer] of
// the sphere (exact where the search box does not cover the axis; the whole
// row otherwise) and split in two where it wraps.  Sets [first, end) of
// sorted records (empty if the row holds no such cell).
__device__ __forceinline__ void wide_run(const Grid &G, const int *start, int r, int ny, int nz,
                                         int cx, int cy, int cz, double fx_, double fy_,
                                         double fz_, const int k[3], const double R[2],
                                         int &first, int &end) {
  const int nc0 = G.nc[0], nc1 = G.nc[1], nc2 = G.nc[2];
  const int part = r & 1;
  int q = r >> 1;
  const int iy = q % ny;
  q /= ny;
  const int iz = q % nz;
  const int layer = q / nz;
  first = end = 0;
  const bool fx = 2 * k[0] + 1 >= nc0, fy = 2 * k[1] + 1 >= nc1, fz = 2 * k[2] + 1 >= nc2;
  const double eta0 = 1e-9 * G.h[0], eta1 = 1e-9 * G.h[1], eta2 = 1e-9 * G.h[2];
  const int oy = iy - k[1], oz = iz - k[2];
  const double gy = fy ? 0.0 : face_gap(oy, fy_, G.h[1], eta1);
  const double gz = fz ? 0.0 : face_gap(oz, fz_, G.h[2], eta2);
  const double Rl = R[layer];
  const double rest = Rl * Rl - (gy * gy + gz * gz);
  if (!(rest >= 0.0)) return;
  const int z = fz ? iz : (cz + oz + nc2) % nc2;
  const int y = fy ? iy : (cy + oy + nc1) % nc1;
  const int row = (layer ? G.layer2 : 0) + (z * nc1 + y) * nc0;
  int xa = 0, xb = 0;  // cells [xa, xb) of the row, in offsets when not wrapping the axis
  if (fx) {
    if (!part) xb = nc0;
  } else {
    // x offsets whose cells come within the remaining distance
    const double ext = __builtin_sqrt(rest) * (1.0 + 1e-9) + eta0;
    int o0 = -k[0], o1 = k[0];
    while (o0 < 0 && face_gap(o0, fx_, G.h[0], 0.0) > ext) ++o0;
    while (o1 > 0 && face_gap(o1, fx_, G.h[0], 0.0) > ext) --o1;
    const int x0 = cx + o0, x1 = cx + o1;
    if (x0 < 0) {
      xa = part ? 0 : x0 + nc0;
      xb = part ? x1 + 1 : nc0;
    } else if (x1 >= nc0) {
      xa = part ? 0 : x0;
      xb = part ? x1 - nc0 + 1 : nc0;
    } else if (!part) {
      xa = x0;
      xb = x1 + 1;
    }
  }
  if (xb > xa) {
    first = start[row + xa];
    end = start[row + xb];
  }
}

// a5 for the spheres of large extent (second layer of a split grid): one wave
// per sphere p tests every sphere that can touch it exactly (rule 1 with the
// canonical minimum image): of the first layer, those within p's extent plus
// rho_c (their extents are at most rho_c); of the second layer, those after p
// within p's extent plus the largest extent, so each pair of large-extent
// spheres is tested once.  Pairs of two first-layer spheres belong to
// k_detect_half.  The lanes first fetch up to 64 row runs of the ball-pruned
// search box at once and scan their lengths; then each lane takes every 64th
// candidate of the concatenated runs, finding its run by a binary search over
// the scanned lengths held across the wave.  An FMA pre-filter (tolerance for
// the full reach) keeps the exact rule for the few pairs that may touch;
// survivors are decided at once (they are rare).
__global__ __launch_bounds__(256) void k_detect_wide(DetectArgs A, const int *first_dev, int n) {
  const int first = *first_dev, count = n - first;
  const int lane = __lane_id();
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = (gridDim.x * blockDim.x) / WAVE;
  const Grid &G = A.G;
  unsigned long long tests = 0ull;
  for (int w = wid; w < count; w += nw) {
    const int p = first + w;
    const Rec a = A.rec[p];
    const double ea = extent(a.r, a.vx, a.vy, a.vz, A.dt);
    const double R[2] = {(ea + A.rho_c) * (1.0 + 1e-9), (ea + G.rho_max) * (1.0 + 1e-9)};
    int k[3];
    for (int ax = 0; ax < 3; ++ax) k[ax] = (int)ceil(R[1] / G.h[ax]);
    const int cx = cell_coord(a.x, G.inv_h[0], G.nc[0]);
    const int cy = cell_coord(a.y, G.inv_h[1], G.nc[1]);
    const int cz = cell_coord(a.z, G.inv_h[2], G.nc[2]);
    const double fx_ = a.x - cx * G.h[0], fy_ = a.y - cy * G.h[1], fz_ = a.z - cz * G.h[2];
    const int ny = 2 * k[1] + 1 >= G.nc[1] ? G.nc[1] : 2 * k[1] + 1;
    const int nz = 2 * k[2] + 1 >= G.nc[2] ? G.nc[2] : 2 * k[2] + 1;
    const int nruns = 2 * 2 * ny * nz;
    for (int rb = 0; rb < nruns; rb += WAVE) {
      int s0 = 0, s1 = 0;
      if (rb + lane < nruns) {
        wide_run(G, A.start, rb + lane, ny, nz, cx, cy, cz, fx_, fy_, fz_, k, R, s0, s1);
        if ((((rb + lane) >> 1) / (ny * nz)) == 1) {  // second layer: only j after p
          s0 = s0 > p + 1 ? s0 : p + 1;
          s1 = s1 > s0 ? s1 : s0;
        }
      }
      const int len = s1 - s0;
      int incl = len;
      for (int o = 1; o < WAVE; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
      }
      const int excl = incl - len;
      const int total = __shfl(incl, WAVE - 1);
      for (int base = 0; base < total; base += WAVE) {
        const int v = base + lane;
        // largest lane l with excl[l] <= v: the run holding candidate v
        int l = 0;
        for (int step = WAVE / 2; step > 0; step >>= 1) {
          const int c = l + step;
          const int ec = __shfl(excl, c);
          if (ec <= v) l = c;
        }
        const int j = __shfl(s0, l) + (v - __shfl(excl, l));
        if (v < total) {
          ++tests;
          const Rec b = A.rec[j];
          const double d0 = wrap_sep(b.x - a.x, G.L[0], G.halfL[0]);
          const double d1 = wrap_sep(b.y - a.y, G.L[1], G.halfL[1]);
          const double d2 = wrap_sep(b.z - a.z, G.L[2], G.halfL[2]);
          const double u0 = b.vx - a.vx, u1 = b.vy - a.vy, u2 = b.vz - a.vz;
          const double s = a.r + b.r;
          const double bf = __builtin_fma(d0, u0, __builtin_fma(d1, u1, d2 * u2));
          const double cf =
              __builtin_fma(d0, d0, __builtin_fma(d1, d1, __builtin_fma(d2, d2, -(s * s))));
          double t;
          if (__builtin_fma(bf, A.dt2, cf) <= A.tol_wide &&
              contact_time(d0, d1, d2, u0, u1, u2, s, A.dt, t))
            record_contact(A, p, j, t);
        }
      }
    }
  }
  block_add(tests, &my_shard(A.ctr).tests);
}

hipError_t launch_detect_wide(hipStream_t s, const DetectArgs &A, const int *first_dev, int n) {
  if (n <= 0) return hipSuccess;
  // the range is on the device (no read-back before the launch): waves loop
  // over it; about one wave per 256 spheres (the split puts about 0.1% of them
  // in the second layer), 64 to 4096
  int64_t waves = n / 256;
  waves = waves < 64 ? 64 : (waves > 4096 ? 4096 : waves);
  hipLaunchKernelGGL(k_detect_wide, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, A,
                     first_dev, n);
  return hipGetLastError();
}

// Earliest partner (rule 2: exact binary64 t, ties to the smaller caller index;
// with crank given, the contact of smallest curve rank) by an exact search of
// the sphere's search box (the 27 surrounding cells, or the wider box of a
// split grid, in both layers), minimum image by rule 1.
// One wave per sphere; lanes over candidates; the wave reduces (t, caller
// index) exactly.  Spheres come from `list` (length nlist, or *nlist_dev when
// given) or, with list NULL, are all i < nlist whose status is `select`
// (select < 0: all); selected DIRTY spheres become ACTIVE.  Collided spheres
// are never candidates.  Used for spheres whose contacts overflowed the slots,
// for pcol_detect with an active mask, and for grids with fewer than 3 cells
// along some axis.
__global__ __launch_bounds__(256) void k_gather_exact(const int *list, int nlist,
                                                      const unsigned int *nlist_dev, int select,
                                                      const Rec *rec, const int *start, Grid G0,
                                                      double dt, uint8_t *status, int *key_j,
                                                      double *key_t, BatchDev B,
                                                      const unsigned long long *crank) {
  if (B.flags && (B.flags[FLAG_ERR] || B.flags[FLAG_DONE])) return;
  const int lane = __lane_id();
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = (gridDim.x * blockDim.x) / WAVE;
  const int count = nlist_dev ? (int)*nlist_dev : nlist;
  for (int w = wid; w < count; w += nw) {
    const int i = list ? list[w] : w;
    if (select >= 0 && status[i] != (uint8_t)select) continue;
    // the sphere's grid: the single one, or its box's in the batched form
    const Rec a = rec[i];
    const int bx = B.gtab ? a.box : 0;
    const Grid G = B.gtab ? B.gtab[bx] : G0;
    const int *st = B.gtab ? start + B.cell_base[bx] : start;
    int k[3];
    search_radius(G, a, dt, k);
    const int cx = cell_coord(a.x, G.inv_h[0], G.nc[0]);
    const int cy = cell_coord(a.y, G.inv_h[1], G.nc[1]);
    const int cz = cell_coord(a.z, G.inv_h[2], G.nc[2]);
    double bt = INFINITY;
    int bo = 0x7fffffff, bj = -1;
    unsigned long long br = ~0ull;  // literal order: curve rank of the best contact
    for (int layer = 0; layer < (G.layer2 ? 2 : 1); ++layer) {
      search_box_runs(G, st, layer ? G.layer2 : 0, cx, cy, cz, k, [&](int s0, int s1) {
        for (int j = s0 + lane; j < s1; j += WAVE) {
          if (j == i) continue;
          if (status[j] == ST_COLLIDED) continue;
          const Rec b = rec[j];
          double t;
          if (pair_time_walls(a, b, G, dt, t)) {
            const int o = b.o;
            if (crank) {
              const unsigned long long rj = crank[j];
              if (rj < br) {
                br = rj;
                bt = t;
                bj = j;
              }
            } else if (t < bt || (t == bt && o < bo)) {
              bt = t;
              bo = o;
              bj = j;
            }
          }
        }
      });
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const double t2 = __shfl_xor(bt, o);
      const int o2 = __shfl_xor(bo, o);
      const int j2 = __shfl_xor(bj, o);
      const unsigned long long r2 = __shfl_xor(br, o);
      if (crank ? r2 < br : (t2 < bt || (t2 == bt && o2 < bo))) {
        bt = t2;
        bo = o2;
        bj = j2;
        br = r2;
      }
    }
    if (lane == 0) {
      key_j[i] = bj;
      key_t[i] = bt;
      if (status[i] == ST_DIRTY) status[i] = ST_ACTIVE;
    }
  }
}

hipError_t launch_gather_exact(hipStream_t s, const int *list, int nlist, const unsigned int *nlist_dev,
                               int select, const Rec *rec, const int *start, const Grid &G,
                               double dt, uint8_t *status, int *key_j, double *key_t,
                               const BatchDev *B, const unsigned long long *crank) {
  int64_t waves = nlist_dev ? 8192 : nlist;
  if (waves <= 0) return hipSuccess;
  if (waves > 8192) waves = 8192;
  const int blocks = (int)((waves + 3) / 4);
  BatchDev none{};
  hipLaunchKernelGGL(k_gather_exact, dim3(blocks), dim3(256), 0, s, list, nlist, nlist_dev, select,
                     rec, start, G, dt, status, key_j, key_t, B ? *B : none, crank);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a6: mutual resolve

// One sweep of rule 3-4 over every ACTIVE sphere (cell-sorted order).  A sphere
// whose partner has it as partner resolves its own side of the pair from the
// start-of-step records and writes its end-of-step state to its output record
// (Sec. "Inter-Particle Collisions"; eq. update_vel, update_rho).  A sphere
// whose partner pairs with a third sphere this sweep becomes DIRTY (new partner
// search next sweep); one without a partner becomes FREE for the step.  Each
// thread writes only its own status, and reads only keys, so the sweep is a
// pure function of the keys.  Partners are spatial neighbours, so the partner
// reads stay within a few cells of the sorted order.
// SPIN: the friction-and-spin resolve (S given); the plain kernel leaves it out
// and needs half the registers, which the sweeps' random reads repay in waves.
template <bool SPIN>
__global__ __launch_bounds__(256) void k_resolve_sweep(int n, const Rec *rec, Grid G0, double dt,
                                                       double e, const double *mass,
                                                       const int *key_j, const double *key_t,
                                                       uint8_t *status, OutRec *out,
                                                       SweepCounters *ctr, BatchDev B,
                                                       const int *list,
                                                       int nlist, Spin S) {
  if (B.flags && (B.flags[FLAG_ERR] || B.flags[FLAG_DONE])) return;
  const int ti = blockIdx.x * 256 + threadIdx.x;
  const bool valid = list ? ti < nlist : ti < n;
  const int i = list && valid ? list[ti] : ti;
  unsigned long long npair = 0ull;
  if (valid && status[i] == ST_ACTIVE) {
    const int p = key_j[i];
    if (p < 0) {
      status[i] = ST_FREE;
    } else {
      const int q = key_j[p];
      if (SPIN && q == i) {
        // with spins, the thread of the smaller sorted index resolves both sides
        // and writes both spins in place (the partner's thread writes nothing,
        // so no thread reads a spin another one has already changed)
        if (i < p) {
          const Rec a = rec[i], b = rec[p];
          const double t = key_t[i];
          const double ma = mass[a.o], mb = mass[b.o];
          const double wa[3] = {S.wx[a.o], S.wy[a.o], S.wz[a.o]};
          const double wb[3] = {S.wx[b.o], S.wy[b.o], S.wz[b.o]};
          double xo[3], vo[3], wo[3];
          resolve_one_spin(a, b, ma, mb, wa, wb, G0, t, dt, e, S.mu, xo, vo, wo);
          out[i] = OutRec{xo[0], xo[1], xo[2], vo[0], vo[1], vo[2], t, b.o, 0u};
          S.wx[a.o] = wo[0];
          S.wy[a.o] = wo[1];
          S.wz[a.o] = wo[2];
          resolve_one_spin(b, a, mb, ma, wb, wa, G0, t, dt, e, S.mu, xo, vo, wo);
          out[p] = OutRec{xo[0], xo[1], xo[2], vo[0], vo[1], vo[2], t, a.o, 0u};
          S.wx[b.o] = wo[0];
          S.wy[b.o] = wo[1];
          S.wz[b.o] = wo[2];
          status[i] = ST_COLLIDED;
          status[p] = ST_COLLIDED;
          npair = 1ull;
        }
      } else if (q == i) {
        const Rec a = rec[i], b = rec[p];
        const double t = key_t[i];
        const double ma = mass[a.o], mb = mass[b.o];
        double xo[3], vo[3];
        if (B.gtab) {
          const Grid G = B.gtab[a.box];
          resolve_one(a, b, ma, mb, G, t, dt, e, xo, vo);
        } else {
          resolve_one(a, b, ma, mb, G0, t, dt, e, xo, vo);
        }
        OutRec o;
        o.x = xo[0];
        o.y = xo[1];
        o.z = xo[2];
        o.vx = vo[0];
        o.vy = vo[1];
        o.vz = vo[2];
        o.t = t;
        o.partner = b.o;
        o.pad = 0u;
        out[i] = o;
        status[i] = ST_COLLIDED;
        if (i < p) npair = 1ull;
      } else if (q >= 0 && key_j[q] == p) {
        status[i] = ST_DIRTY;  // p pairs with q this sweep
      }
    }
  }
  block_add(npair, &my_shard(ctr).pairs);
}

hipError_t launch_resolve_sweep(hipStream_t s, int n, const Rec *rec, const Grid &G, double dt,
                                double e, const double *mass, const int *key_j,
                                const double *key_t, uint8_t *status, OutRec *out,
                                SweepCounters *ctr, const BatchDev *B,
                                const int *list, int nlist, const Spin *spin) {
  const int items = list ? nlist : n;
  if (items <= 0) return hipSuccess;
  BatchDev none{};
  if (spin && spin->wx)
    hipLaunchKernelGGL(k_resolve_sweep<true>, dim3((items + 255) / 256), dim3(256), 0, s, n, rec,
                       G, dt, e, mass, key_j, key_t, status, out, ctr, B ? *B : none, list, nlist,
                       *spin);
  else
    hipLaunchKernelGGL(k_resolve_sweep<false>, dim3((items + 255) / 256), dim3(256), 0, s, n, rec,
                       G, dt, e, mass, key_j, key_t, status, out, ctr, B ? *B : none, list, nlist,
                       Spin{nullptr, nullptr, nullptr, 0.0});
  return hipGetLastError();
}

// The spheres a sweep left ACTIVE or DIRTY, in sorted order, as a list for the
// later sweeps (the others are done for the step): per-workgroup counts, an
// exclusive scan of the counts (launch_scan), then each workgroup writes its
// spheres from its offset.  No shared counter.
__global__ __launch_bounds__(256) void k_keep_count(const uint8_t *status, int n, int *count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && (status[i] == ST_ACTIVE || status[i] == ST_DIRTY);
  __shared__ int part[256 / WAVE];
  const int c = __popcll(__ballot(keep));
  if (__lane_id() == 0) part[threadIdx.x / WAVE] = c;
  __syncthreads();
  if (threadIdx.x == 0) count[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ __launch_bounds__(256) void k_keep_write(const uint8_t *status, int n, const int *off,
                                                    int *list) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && (status[i] == ST_ACTIVE || status[i] == ST_DIRTY);
  __shared__ int part[256 / WAVE];
  const unsigned long long m = __ballot(keep);
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0) part[w] = __popcll(m);
  __syncthreads();
  int base = off[blockIdx.x];
  for (int k = 0; k < w; ++k) base += part[k];
  if (keep) list[base + __popcll(m & ((1ull << __lane_id()) - 1ull))] = i;
}

hipError_t launch_keep_list(hipStream_t s, const uint8_t *status, int n, int *count, int *off,
                            int *blocksum, ReachOut *scratch_out, int *list) {
  if (n <= 0) return hipSuccess;
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_keep_count, dim3(nb), dim3(256), 0, s, status, n, count);
  hipError_t e = launch_scan(s, count, nb, off, blocksum, scratch_out);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_keep_write, dim3(nb), dim3(256), 0, s, status, n, off, list);
  return hipGetLastError();
}

// a8 and the copy back: the end-of-step state of every sphere in the caller's
// order (coalesced writes).  A sphere whose status (sorted order) says it
// collided this step takes the output record its resolve wrote; any other
// flies the whole step from its start state, still in the caller's arrays
// (rule 5).  Only collided spheres read their 64-B output record; the others
// read one status byte (a 1-B-per-sphere array that stays in the device's
// last-level cache).
__global__ __launch_bounds__(256) void k_finish(Particles P, const int *rank,
                                                const OutRec *out, const uint8_t *status,
                                                int *partner, double *tcoll, double dt, Grid G0,
                                                BatchDev B) {
  if (B.flags && (B.flags[FLAG_ERR] || B.flags[FLAG_UNFINISHED])) return;
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= P.n) return;
  double x, y, z, vx, vy, vz, t;
  int pj;
  const int q = rank[o];
  if (status[q] == ST_COLLIDED) {
    const OutRec r = out[q];
    x = r.x;
    y = r.y;
    z = r.z;
    vx = r.vx;
    vy = r.vy;
    vz = r.vz;
    t = r.t;
    pj = r.partner;
  } else {
    const double *L = B.gtab ? B.gtab[B.box_of[o]].L : G0.L;
    const int walls = B.gtab ? 0 : G0.walls;  // the batched form has periodic boxes only
    vx = P.vx[o];
    vy = P.vy[o];
    vz = P.vz[o];
    x = fly_axis(P.x[o] + dt * vx, L[0], walls & 1, vx);
    y = fly_axis(P.y[o] + dt * vy, L[1], walls & 2, vy);
    z = fly_axis(P.z[o] + dt * vz, L[2], walls & 4, vz);
    t = __longlong_as_double(0x7ff8000000000000LL);  // NaN: no collision
    pj = -1;
  }
  P.x[o] = x;
  P.y[o] = y;
  P.z[o] = z;
  P.vx[o] = vx;
  P.vy[o] = vy;
  P.vz[o] = vz;
  partner[o] = pj;
  tcoll[o] = t;
}

hipError_t launch_finish(hipStream_t s, const Particles &P, const int *rank, const OutRec *out,
                         const uint8_t *status, int *partner, double *tcoll, double dt,
                         const Grid &G, const BatchDev *B) {
  if (P.n <= 0) return hipSuccess;
  BatchDev none{};
  hipLaunchKernelGGL(k_finish, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s, P, rank, out,
                     status, partner, tcoll, dt, G, B ? *B : none);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a8: free flight + wrap

// rule 5: spheres that did not collide fly the whole step; coalesced over the
// caller's order.
__global__ __launch_bounds__(256) void k_advance(Particles P, const int *partner, double dt,
                                                 double L0, double L1, double L2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= P.n || partner[i] >= 0) return;
  P.x[i] = wrap_pos(P.x[i] + dt * P.vx[i], L0);
  P.y[i] = wrap_pos(P.y[i] + dt * P.vy[i], L1);
  P.z[i] = wrap_pos(P.z[i] + dt * P.vz[i], L2);
}

hipError_t launch_advance(hipStream_t s, const Particles &P, const int *partner, double dt,
                          const double L[3]) {
  if (P.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_advance, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s, P, partner,
                     dt, L[0], L[1], L[2]);
  return hipGetLastError();
}

// ---------------------------------------------------------------- public single-sweep API

// caller active mask -> sorted status (inactive spheres are excluded like
// collided ones)
__global__ __launch_bounds__(256) void k_status_from_active(const uint8_t *active,
                                                            const Rec *rec, int n,
                                                            uint8_t *status) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  status[i] = (active ? active[rec[i].o] != 0 : true) ? ST_ACTIVE : ST_COLLIDED;
}

hipError_t launch_status_from_active(hipStream_t s, const uint8_t *active, const Rec *rec, int n,
                                     uint8_t *status) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_status_from_active, dim3((n + 255) / 256), dim3(256), 0, s, active, rec,
                     n, status);
  return hipGetLastError();
}

// keys in the caller's order: (bits of (float)t) << 32 | caller index of the partner
__global__ __launch_bounds__(256) void k_export_keys(int n, const Rec *rec, const int *key_j,
                                                     const double *key_t, const uint8_t *status,
                                                     uint64_t *key_out, double *tmin_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int o = rec[i].o;
  const int j = key_j[i];
  const bool has = j >= 0 && (!status || status[i] == ST_ACTIVE);
  uint64_t key = ~0ull;
  double t = INFINITY;
  if (has) {
    t = key_t[i];
    const float tf = (float)t;
    key = ((uint64_t)__float_as_uint(tf) << 32) | (uint64_t)(uint32_t)rec[j].o;
  }
  key_out[o] = key;
  if (tmin_out) tmin_out[o] = t;
}

hipError_t launch_export_keys(hipStream_t s, int n, const Rec *rec, const int *key_j,
                              const double *key_t, const uint8_t *status, uint64_t *key_out,
                              double *tmin_out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_keys, dim3((n + 255) / 256), dim3(256), 0, s, n, rec, key_j, key_t,
                     status, key_out, tmin_out);
  return hipGetLastError();
}

// rule 3-4 from caller-order keys; start-of-step data from the binned records
__global__ __launch_bounds__(256) void k_resolve_public(int n, const Rec *rec, const int *rank,
                                                        Grid G, double dt, double e,
                                                        const uint64_t *key, Particles P,
                                                        uint8_t *active, int *partner,
                                                        double *tcoll, long long *npairs) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  unsigned long long np = 0ull;
  if (i < n && active[i] != 0 && key[i] != ~0ull) {
    const int p = (int)(uint32_t)(key[i] & 0xffffffffull);
    if (p >= 0 && p < n && p != i && key[p] != ~0ull &&
        (int)(uint32_t)(key[p] & 0xffffffffull) == i) {
      const Rec a = rec[rank[i]], b = rec[rank[p]];
      double t;
      if (pair_time(a, b, G, dt, t)) {
        double xo[3], vo[3];
        resolve_one(a, b, P.m[i], P.m[p], G, t, dt, e, xo, vo);
        P.x[i] = xo[0];
        P.y[i] = xo[1];
        P.z[i] = xo[2];
        P.vx[i] = vo[0];
        P.vy[i] = vo[1];
        P.vz[i] = vo[2];
        active[i] = 0;
        if (partner) partner[i] = p;
        if (tcoll) tcoll[i] = t;
        if (i < p) np = 1ull;
      }
    }
  }
  np = wave_sum(np);
  if (__lane_id() == 0 && np && npairs) atomicAdd((unsigned long long *)npairs, np);
}

hipError_t launch_resolve_public(hipStream_t s, int n, const Rec *rec, const int *rank,
                                 const Grid &G, double dt, double e, const uint64_t *key,
                                 const Particles &P, uint8_t *active, int *partner, double *tcoll,
                                 long long *npairs) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resolve_public, dim3((n + 255) / 256), dim3(256), 0, s, n, rec, rank, G,
                     dt, e, key, P, active, partner, tcoll, npairs);
  return hipGetLastError();
}

}  // namespace pcol

namespace pcol {

// ---------------------------------------------------------------- adjoint of one step

// Reverse-mode derivative of one step with the pair set fixed (caller order).
// Forward quantities of a pair (i, j) from i's side, as in resolve_one:
//   d = x_j - x_i (minimum image), u = v_j - v_i, t = contact time, w = d + t u,
//   n = w / s, g = u . n, c = m_r (1 + e), J = c g,
//   vi' = v_i + (J/m_i) n,  vj' = v_j - (J/m_j) n,
//   xi' = x_i + t v_i + (dt - t) vi',  xj' = x_j + t v_j + (dt - t) vj'.
// The contact time depends on (d, u) through |d + t u| = s:  dt/dd = -n/g,
// dt/du = -t n/g.  Given the gradients G of the loss with respect to the
// end-of-step state of i and j, the sweep of adjoints below returns the
// gradient with respect to i's start state; each thread writes only its own
// sphere, and the e-gradient of the pair is stored once (by the smaller index).
// Spheres without a collision: x' = x + dt v gives gx = Gx, gv = Gv + dt Gx.
__global__ __launch_bounds__(256) void k_step_backward(int n, const double *x, const double *y,
                                                       const double *z, const double *vx,
                                                       const double *vy, const double *vz,
                                                       const double *r, const double *m, Grid G,
                                                       double dt, double e, const int *partner,
                                                       const double *tcoll, StateGrad gout,
                                                       StateGrad gin, double *ebuf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = partner[i];
  const double Gxi[3] = {gout.x[i], gout.y[i], gout.z[i]};
  const double Gvi[3] = {gout.vx[i], gout.vy[i], gout.vz[i]};
  if (j < 0) {
    gin.x[i] = Gxi[0];
    gin.y[i] = Gxi[1];
    gin.z[i] = Gxi[2];
    gin.vx[i] = Gvi[0] + dt * Gxi[0];
    gin.vy[i] = Gvi[1] + dt * Gxi[1];
    gin.vz[i] = Gvi[2] + dt * Gxi[2];
    ebuf[i] = 0.0;
    return;
  }
  const double Gxj[3] = {gout.x[j], gout.y[j], gout.z[j]};
  const double Gvj[3] = {gout.vx[j], gout.vy[j], gout.vz[j]};
  const double xi[3] = {x[i], y[i], z[i]}, xj[3] = {x[j], y[j], z[j]};
  const double vi[3] = {vx[i], vy[i], vz[i]}, vj[3] = {vx[j], vy[j], vz[j]};
  const double t = tcoll[i];
  double d[3], u[3], nn[3];
  for (int k = 0; k < 3; ++k) {
    d[k] = wrap_sep(xj[k] - xi[k], G.L[k], G.halfL[k]);
    u[k] = vj[k] - vi[k];
  }
  const double s = r[i] + r[j];
  for (int k = 0; k < 3; ++k) nn[k] = (d[k] + t * u[k]) / s;
  const double g = (u[0] * nn[0] + u[1] * nn[1]) + u[2] * nn[2];
  const double mr = (m[i] * m[j]) / (m[i] + m[j]);
  const double c = mr * (1.0 + e);
  const double J = c * g;
  double vin[3], vjn[3];
  for (int k = 0; k < 3; ++k) {
    vin[k] = vi[k] + (J / m[i]) * nn[k];
    vjn[k] = vj[k] - (J / m[j]) * nn[k];
  }
  // adjoints
  double tb = 0.0, Jb = 0.0, bvi[3], bvj[3], bvin[3], bvjn[3], bn[3], bu[3], bd[3];
  for (int k = 0; k < 3; ++k) {
    tb += Gxi[k] * (vi[k] - vin[k]) + Gxj[k] * (vj[k] - vjn[k]);
    bvin[k] = Gvi[k] + (dt - t) * Gxi[k];
    bvjn[k] = Gvj[k] + (dt - t) * Gxj[k];
    bvi[k] = t * Gxi[k] + bvin[k];
    bvj[k] = t * Gxj[k] + bvjn[k];
    Jb += bvin[k] * nn[k] / m[i] - bvjn[k] * nn[k] / m[j];
    bn[k] = (J / m[i]) * bvin[k] - (J / m[j]) * bvjn[k];
  }
  const double gb = c * Jb;
  const double eb = mr * g * Jb;
  for (int k = 0; k < 3; ++k) {
    bu[k] = gb * nn[k];
    bn[k] += gb * u[k];
  }
  double wb[3];
  for (int k = 0; k < 3; ++k) {
    wb[k] = bn[k] / s;
    bd[k] = wb[k];
    tb += wb[k] * u[k];
    bu[k] += t * wb[k];
  }
  for (int k = 0; k < 3; ++k) {
    bd[k] += (-tb / g) * nn[k];
    bu[k] += (-tb * t / g) * nn[k];
  }
  // d = x_j - x_i, u = v_j - v_i
  gin.x[i] = Gxi[0] - bd[0];
  gin.y[i] = Gxi[1] - bd[1];
  gin.z[i] = Gxi[2] - bd[2];
  gin.vx[i] = bvi[0] - bu[0];
  gin.vy[i] = bvi[1] - bu[1];
  gin.vz[i] = bvi[2] - bu[2];
  (void)bvj;
  ebuf[i] = i < j ? eb : 0.0;
}

// deterministic sum of v[0..n) (fixed tree order) added to *out; one block
__global__ __launch_bounds__(1024) void k_sum_det(const double *v, int n, double *out) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 1024) acc += v[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out += part[0];
}

hipError_t launch_step_backward(hipStream_t s, const Particles &P, const Grid &G, double dt,
                                double e, const int *partner, const double *tcoll,
                                const StateGrad &gout, const StateGrad &gin, double *ebuf,
                                double *ge) {
  const int n = (int)P.n;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step_backward, dim3((n + 255) / 256), dim3(256), 0, s, n, P.x, P.y, P.z,
                     P.vx, P.vy, P.vz, P.r, P.m, G, dt, e, partner, tcoll, gout, gin, ebuf);
  hipLaunchKernelGGL(k_sum_det, dim3(1), dim3(1024), 0, s, ebuf, n, ge);
  return hipGetLastError();
}

}  // namespace pcol

namespace pcol {

// ---------------------------------------------------------------- batched form

// box id of every sphere (caller order), one workgroup per box
__global__ __launch_bounds__(256) void k_fill_box_of(const int64_t *box_off, int *box_of) {
  const int b = blockIdx.x;
  for (int64_t i = box_off[b] + threadIdx.x; i < box_off[b + 1]; i += 256) box_of[i] = b;
}

hipError_t launch_fill_box_of(hipStream_t s, int nbox, const int64_t *box_off, int *box_of) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_box_of, dim3(nbox), dim3(256), 0, s, box_off, box_of);
  return hipGetLastError();
}

// a1 per box: data validity, reach = 2 max r + 2 max|v| dt (stored), the box
// check L > 2 reach, and whether the planned cells are still at least the reach
// wide (else the host re-plans before any state changes).  Boxes are cut into
// chunks of at most BREACH_CHUNK spheres, one workgroup each, which merge their
// maxima into the box's BoxMax; k_breach_fin then takes one box per thread
// and clears its BoxMax for the next pass.
// BIN: the same pass also takes each sphere's global cell (the box's first
// cell + its cell on the box's planned grid) and its slot in that cell, before
// k_breach_fin has checked the data and the plan: cell coordinates are
// clamped, so every count stays inside the plan's cells, and a failed check
// stops every kernel after it.
template <bool BIN>
__global__ __launch_bounds__(256) void k_breach(Particles P, BatchDev B, int *cid, int *slot,
                                                int *count) {
  const int b = B.chunk_box[blockIdx.x];
  const Grid &G = B.gtab[b];
  const int64_t lo = B.chunk_lo[blockIdx.x];
  const int64_t hi = lo + BREACH_CHUNK < B.box_off[b + 1] ? lo + BREACH_CHUNK : B.box_off[b + 1];
  double v2 = 0.0, rm = 0.0;
  unsigned int bad = 0u;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double x = P.x[i], y = P.y[i], z = P.z[i];
    const double vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
    const double r = P.r[i], m = P.m[i];
    const double w = (vx * vx + vy * vy) + vz * vz;
    const bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(w) && isfinite(r) &&
                     isfinite(m);
    if (!fin || !(r > 0.0) || !(m > 0.0)) bad |= ERR_INVALID;
    if (!(x >= 0.0 && x < G.L[0]) || !(y >= 0.0 && y < G.L[1]) || !(z >= 0.0 && z < G.L[2]))
      bad |= ERR_INVALID;
    if (fin) {
      v2 = w > v2 ? w : v2;
      rm = r > rm ? r : rm;
    }
    if (BIN) {
      const int cx = cell_coord(x, G.inv_h[0], G.nc[0]);
      const int cy = cell_coord(y, G.inv_h[1], G.nc[1]);
      const int cz = cell_coord(z, G.inv_h[2], G.nc[2]);
      const int c = B.cell_base[b] + (cz * G.nc[1] + cy) * G.nc[0] + cx;
      cid[i] = c;
      slot[i] = atomicAdd(&count[c], 1);
    }
  }
  __shared__ double sv[4], sr[4];
  __shared__ unsigned int sb[4];
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double a = __shfl_xor(v2, o), c = __shfl_xor(rm, o);
    v2 = a > v2 ? a : v2;
    rm = c > rm ? c : rm;
    bad |= __shfl_xor(bad, o);
  }
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0) {
    sv[w] = v2;
    sr[w] = rm;
    sb[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      v2 = sv[k] > v2 ? sv[k] : v2;
      rm = sr[k] > rm ? sr[k] : rm;
      bad |= sb[k];
    }
    atomicMax(&B.bmax[b].v2, dbits(v2));
    atomicMax(&B.bmax[b].rm, dbits(rm));
    if (bad) atomicOr(&B.bmax[b].bad, bad);
  }
}

__global__ __launch_bounds__(256) void k_breach_fin(BatchDev B, double dt, int check_plan) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B.nbox) return;
  const BoxMax mx = B.bmax[b];
  B.bmax[b] = BoxMax{0ull, 0ull, 0u, 0u};
  const double v2 = __longlong_as_double((long long)mx.v2);
  const double rm = __longlong_as_double((long long)mx.rm);
  unsigned int bad = mx.bad;
  const Grid &G = B.gtab[b];
  const double reach = 2.0 * rm + 2.0 * sqrt(v2) * dt;
  B.breach[b] = reach;
  for (int a = 0; a < 3; ++a) {
    if (!(G.L[a] > 2.0 * reach)) bad |= ERR_BOX;
    if (check_plan && !(reach * (1.0 + 1e-9) <= G.L[a] / G.nc[a])) bad |= ERR_REPLAN;
  }
  if (bad) atomicOr(&B.flags[FLAG_ERR], bad);
}

hipError_t launch_breach(hipStream_t s, const Particles &P, const BatchDev &B, double dt,
                         int check_plan, int *cid, int *slot, int *count) {
  if (B.nbox <= 0) return hipSuccess;
  if (B.nchunk > 0) {
    if (count)
      hipLaunchKernelGGL(k_breach<true>, dim3(B.nchunk), dim3(256), 0, s, P, B, cid, slot, count);
    else
      hipLaunchKernelGGL(k_breach<false>, dim3(B.nchunk), dim3(256), 0, s, P, B, nullptr, nullptr,
                         nullptr);
  }
  hipLaunchKernelGGL(k_breach_fin, dim3((B.nbox + 255) / 256), dim3(256), 0, s, B, dt, check_plan);
  return hipGetLastError();
}

hipError_t launch_detect_batched(hipStream_t s, const DetectArgs &A, const BatchDev &B,
                                 int total_cells, int cpw) {
  if (cpw < 1 || total_cells <= 0) return cpw < 1 ? hipErrorInvalidValue : hipSuccess;
  hipLaunchKernelGGL(k_detect_batched, dim3((unsigned)((total_cells + cpw - 1) / cpw)), dim3(WAVE),
                     0, s, A, B, cpw);
  return hipGetLastError();
}

// After a sweep's resolve: total the pairs it resolved (and the running totals),
// clear the per-sweep counters, and mark the step done when the sweep resolved
// none.  `last` marks the final sweep slot of a captured step: if pairs were
// still resolved there, the step is unfinished and the host completes it.
__global__ __launch_bounds__(64) void k_sweep_check(SweepCounters *ctr, unsigned int *flags,
                                                    unsigned long long *totals, int last) {
  if (flags[FLAG_ERR] || flags[FLAG_DONE]) return;
  const int l = threadIdx.x;
  unsigned long long p = ctr->shard[l].pairs, c = ctr->shard[l].contacts;
  ctr->shard[l].pairs = 0ull;
  ctr->shard[l].contacts = 0ull;
  p = wave_sum(p);
  c = wave_sum(c);
  if (l == 0) {
    totals[0] += p;
    totals[1] += c;
    totals[2] += ctr->n_overflow;
    ctr->n_overflow = 0u;
    flags[FLAG_SWEEPS] += 1u;
    if (p == 0ull) {
      flags[FLAG_DONE] = 1u;
    } else if (last) {
      flags[FLAG_UNFINISHED] = 1u;
    }
  }
}

hipError_t launch_sweep_check(hipStream_t s, SweepCounters *ctr, unsigned int *flags,
                              unsigned long long *totals, int last) {
  hipLaunchKernelGGL(k_sweep_check, dim3(1), dim3(64), 0, s, ctr, flags, totals, last);
  return hipGetLastError();
}

}  // namespace pcol

// ---------------------------------------------------------------- deposition
//
// Sec. "Dispersed Phase" (projection operator) and Sec. "Deposition": each
// sphere's source components are imposed linearly on the eight corner nodes of
// its host cell of a periodic Cartesian grid (deposition radius = cell side;
// on equal cells the C0 inverse-distance weights are the trilinear ones), and
// every node receives the sum over spheres.  The paper accumulates with atomic
// adds; on this GPU FP64 atomics to HBM run at about 23e9 per second, so 32 per
// sphere would bound the operator at 0.7e9 spheres/s whatever the memory
// order.  Instead the spheres are counted and scattered by element (a counting
// sort, one integer atomic per sphere), each element sums its spheres' corner
// contributions in caller-index order, and each node adds the corner sums of
// its eight elements in a fixed order, in the shared memory of the workgroup
// that owns the node's tile: no floating-point atomics, and the result is the
// same bit for bit on every run.  Nodes are stored node-major:
// out[node * comp + q], node = (k nc1 + j) nc0 + i; element e has the node of
// the same number as its corner (0, 0, 0).
namespace pcol {

namespace {

// Members of an element are taken in caller-index order (a selection over the
// element's records) up to DEP_SORT_MAX; a larger element sums in scatter
// order.  Up to DEP_REG members the selection runs on caller indices held in
// registers (an element holds 3.9 spheres on average in the 16M workload).
constexpr int DEP_SORT_MAX = 64;
constexpr int DEP_REG = 16;

template <int COMP>
struct alignas(16) DepRec {
  double p[3];
  double a[COMP];
  long long o;  // caller index
};

// Host cell and local coordinate of p on one axis: s = p / h, c = floor(s)
// (at most nc - 1), f = s - c in [0, 1].
__device__ __forceinline__ int dep_cell(double p, double h, int nc, double &f) {
  const double s = p / h;
  int c = (int)floor(s);
  c = c > nc - 1 ? nc - 1 : c;
  f = s - (double)c;
  return c;
}

// Element of every sphere and its slot among the element's spheres.  A
// position outside [0, L) or not finite raises bit 0 of *flag and is not
// counted (the host reads the flag before anything else runs).  Consecutive
// lanes of one element (spheres stored in element order) take their slots with
// one atomic per run.
__global__ __launch_bounds__(256) void k_dep_count(DepositArgs D, unsigned int *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int e = -1;  // -1: no element (past the end, or a bad position)
  bool bad = false;
  if (i < D.n) {
    const double p0 = D.x[i], p1 = D.y[i], p2 = D.z[i];
    bad = !(p0 >= 0.0 && p0 < D.L[0]) || !(p1 >= 0.0 && p1 < D.L[1]) ||
          !(p2 >= 0.0 && p2 < D.L[2]);
    if (!bad) {
      double f;
      const int c0 = dep_cell(p0, D.h[0], D.nc[0], f);
      const int c1 = dep_cell(p1, D.h[1], D.nc[1], f);
      const int c2 = dep_cell(p2, D.h[2], D.nc[2], f);
      e = (c2 * D.nc[1] + c1) * D.nc[0] + c0;
    }
  }
  const int lane = (int)__lane_id();
  const unsigned long long badm = __ballot(bad);
  if (badm != 0ull && lane == __ffsll((long long)badm) - 1) atomicOr(flag, 1u);
  const int sl = run_slot(e, D.cnt);
  if (e >= 0) {
    D.eid[i] = e;
    D.slot[i] = sl;
  }
}

// one record per sphere at its element-sorted position (caller arrays read
// coalesced)
template <int COMP>
__global__ __launch_bounds__(256) void k_dep_scatter(DepositArgs D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  DepRec<COMP> r;
  r.p[0] = D.x[i];
  r.p[1] = D.y[i];
  r.p[2] = D.z[i];
#pragma unroll
  for (int q = 0; q < COMP; ++q) r.a[q] = D.a[(int64_t)q * D.n + i];
  r.o = i;
  reinterpret_cast<DepRec<COMP> *>(D.rec)[D.start[D.eid[i]] + D.slot[i]] = r;
}

// The eight corner sums of element e's spheres, each a sum in caller-index
// order of w_b a_q with the trilinear weight
// w_b = ((b0 ? f0 : 1 - f0) (b1 ? f1 : 1 - f1)) (b2 ? f2 : 1 - f2).
template <int COMP>
__device__ __forceinline__ void elem_sums(const DepositArgs &D, int64_t e, double (&acc)[8][COMP]) {
  const DepRec<COMP> *R = reinterpret_cast<const DepRec<COMP> *>(D.rec);
  const int m0 = D.start[e], m1 = D.start[e + 1];
  const bool ordered = m1 - m0 <= DEP_SORT_MAX;
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int q = 0; q < COMP; ++q) acc[b][q] = 0.0;
  auto add = [&](const DepRec<COMP> &r) {
    double f0, f1, f2;
    (void)dep_cell(r.p[0], D.h[0], D.nc[0], f0);
    (void)dep_cell(r.p[1], D.h[1], D.nc[1], f1);
    (void)dep_cell(r.p[2], D.h[2], D.nc[2], f2);
    const double g0 = 1.0 - f0, g1 = 1.0 - f1, g2 = 1.0 - f2;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const double w = (((b & 1) ? f0 : g0) * ((b & 2) ? f1 : g1)) * ((b & 4) ? f2 : g2);
#pragma unroll
      for (int q = 0; q < COMP; ++q) acc[b][q] += w * r.a[q];
    }
  };
  const int m = m1 - m0;
  if (m <= DEP_REG) {
    int oreg[DEP_REG];  // caller indices (< 2^31) of the members, in slot order
#pragma unroll
    for (int u = 0; u < DEP_REG; ++u) oreg[u] = u < m ? (int)R[m0 + u].o : 0x7fffffff;
    int last = -1;
    for (int t = 0; t < m; ++t) {  // the next caller index after `last`
      int best = 0x7fffffff, k = 0;
#pragma unroll
      for (int u = 0; u < DEP_REG; ++u) {
        const bool take = oreg[u] > last && oreg[u] < best;
        best = take ? oreg[u] : best;
        k = take ? u : k;
      }
      last = best;
      add(R[m0 + k]);
    }
  } else {
    long long last = -1;
    for (int t = m0; t < m1; ++t) {
      int k = t;
      if (ordered) {  // the next caller index after `last`, read from the records
        long long best = 0x7fffffffffffffffll;
        for (int u = m0; u < m1; ++u) {
          const long long o = R[u].o;
          if (o > last && o < best) {
            best = o;
            k = u;
          }
        }
        last = best;
      }
      add(R[k]);
    }
  }
}

// Node sums over a tile of DEP_TN^3 nodes: node (i, j, k) is corner b of
// element (i - b0, j - b1, k - b2) (periodic), and receives the eight corner
// sums in the order b = 0..7.  One thread per element of the tile's
// (DEP_TN + 1)^3 elements (the tile's own and one layer below it on each axis)
// forms its element's eight corner sums; then, phase b after phase b, every
// element adds its corner-b sum to the tile node it touches (within a phase no
// two elements share a node), so each node's sum is formed in the order b =
// 0..7 from zero, with no atomics and no corner-sum array in memory.  The
// elements of the lower layer are summed by two to eight tiles.
constexpr int DEP_TN = 7, DEP_TE = DEP_TN + 1, DEP_TILE_THREADS = DEP_TE * DEP_TE * DEP_TE;

template <int COMP>
__global__ __launch_bounds__(DEP_TILE_THREADS) void k_dep_tile(DepositArgs D, int ntx, int nty) {
  __shared__ double nacc[DEP_TN * DEP_TN * DEP_TN * COMP];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int i0 = tx * DEP_TN, j0 = ty * DEP_TN, k0 = tz * DEP_TN;
  const int t = threadIdx.x;
  const int ex = t % DEP_TE, ey = (t / DEP_TE) % DEP_TE, ez = t / (DEP_TE * DEP_TE);
  // the element's global cell, one below the tile's first node on each axis
  auto wrap = [](int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); };
  const int gi = wrap(i0 - 1 + ex, D.nc[0]), gj = wrap(j0 - 1 + ey, D.nc[1]),
            gk = wrap(k0 - 1 + ez, D.nc[2]);
  for (int u = t; u < DEP_TN * DEP_TN * DEP_TN * COMP; u += DEP_TILE_THREADS) nacc[u] = 0.0;
  // every element of the tile's box touches a node of the tile, but past the
  // grid's last cell (a partial tile) it has no node to serve
  const bool live = i0 - 1 + ex < D.nc[0] && j0 - 1 + ey < D.nc[1] && k0 - 1 + ez < D.nc[2];
  double acc[8][COMP];
  if (live) {
    elem_sums<COMP>(D, ((int64_t)gk * D.nc[1] + gj) * D.nc[0] + gi, acc);
  } else {
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int q = 0; q < COMP; ++q) acc[b][q] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int nx = ex - 1 + (b & 1), ny = ey - 1 + ((b >> 1) & 1), nz = ez - 1 + ((b >> 2) & 1);
    const bool hit = live && nx >= 0 && nx < DEP_TN && ny >= 0 && ny < DEP_TN && nz >= 0 &&
                     nz < DEP_TN && i0 + nx < D.nc[0] && j0 + ny < D.nc[1] && k0 + nz < D.nc[2];
    if (hit) {
      double *a = nacc + ((nz * DEP_TN + ny) * DEP_TN + nx) * COMP;
#pragma unroll
      for (int q = 0; q < COMP; ++q) a[q] += acc[b][q];
    }
    __syncthreads();
  }
  if (t < DEP_TN * DEP_TN * DEP_TN) {
    const int nx = t % DEP_TN, ny = (t / DEP_TN) % DEP_TN, nz = t / (DEP_TN * DEP_TN);
    if (i0 + nx < D.nc[0] && j0 + ny < D.nc[1] && k0 + nz < D.nc[2]) {
      const int64_t n = ((int64_t)(k0 + nz) * D.nc[1] + (j0 + ny)) * D.nc[0] + (i0 + nx);
#pragma unroll
      for (int q = 0; q < COMP; ++q) D.out[n * COMP + q] = nacc[t * COMP + q];
    }
  }
}

template <int COMP>
hipError_t deposit_sorted(hipStream_t s, const DepositArgs &D) {
  const unsigned gn = (unsigned)((D.n + 255) / 256);
  if (D.n > 0) hipLaunchKernelGGL(k_dep_scatter<COMP>, dim3(gn), dim3(256), 0, s, D);
  const int ntx = (D.nc[0] + DEP_TN - 1) / DEP_TN, nty = (D.nc[1] + DEP_TN - 1) / DEP_TN,
            ntz = (D.nc[2] + DEP_TN - 1) / DEP_TN;
  hipLaunchKernelGGL(k_dep_tile<COMP>, dim3((unsigned)(ntx * nty * ntz)), dim3(DEP_TILE_THREADS),
                     0, s, D, ntx, nty);
  return hipGetLastError();
}

}  // namespace

int64_t deposit_record_bytes(int comp) { return ((int64_t)(4 + comp) * 8 + 15) / 16 * 16; }

hipError_t launch_deposit_count(hipStream_t s, const DepositArgs &D, unsigned int *flag) {
  if (D.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dep_count, dim3((unsigned)((D.n + 255) / 256)), dim3(256), 0, s, D, flag);
  return hipGetLastError();
}

hipError_t launch_deposit(hipStream_t s, const DepositArgs &D) {
  switch (D.comp) {
    case 1: return deposit_sorted<1>(s, D);
    case 2: return deposit_sorted<2>(s, D);
    case 3: return deposit_sorted<3>(s, D);
    case 4: return deposit_sorted<4>(s, D);
    case 5: return deposit_sorted<5>(s, D);
    case 6: return deposit_sorted<6>(s, D);
    case 7: return deposit_sorted<7>(s, D);
    case 8: return deposit_sorted<8>(s, D);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pcol
