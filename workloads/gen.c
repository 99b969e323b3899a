/*
 * Seeded synthetic particle boxes (inputs only; none of the collision
 * method's arithmetic lives here).
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded through
 * splitmix64; uniform doubles from the top 53 bits; standard normals by the
 * Box-Muller transform (both outputs of each draw are used).
 *
 * Positions: random sequential placement (RSA).  Spheres take uniformly random
 * trial points of the periodic box and a trial is accepted only if it overlaps
 * no sphere placed before it (minimum-image centre distance strictly greater
 * than the sum of radii); see wl_rsa for the batched order of trials.  Polydisperse sets are placed in
 * descending radius order, the usual way to reach high volume fractions with
 * RSA; the final storage order is a seeded random permutation so that index
 * and radius are uncorrelated.
 *
 * Overlap tests use a cell grid whose cells hold their spheres contiguously
 * (x, y, z, r packed), so one trial touches 9 contiguous runs of memory.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } wl_rng;

static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static void rng_seed(wl_rng *g, uint64_t seed, uint64_t stream) {
  uint64_t x = seed * 0x100000001B3ULL ^ (stream + 0x632BE59BD9B4E019ULL);
  for (int k = 0; k < 4; ++k) g->s[k] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }

static inline uint64_t rng_next(wl_rng *g) {
  uint64_t *s = g->s;
  const uint64_t out = rotl(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return out;
}

/* uniform in [0, 1) */
static inline double rng_u01(wl_rng *g) { return (double)(rng_next(g) >> 11) * 0x1.0p-53; }

/* standard normals, n of them, Box-Muller */
void wl_normals(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  wl_rng g;
  rng_seed(&g, seed, stream);
  const double two_pi = 6.283185307179586476925286766559;
  int64_t k = 0;
  while (k < n) {
    double u1 = 1.0 - rng_u01(&g); /* (0, 1] */
    double u2 = rng_u01(&g);
    double rad = sqrt(-2.0 * log(u1));
    out[k++] = rad * cos(two_pi * u2);
    if (k < n) out[k++] = rad * sin(two_pi * u2);
  }
}

/* uniforms in [0, 1) */
void wl_uniforms(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  wl_rng g;
  rng_seed(&g, seed, stream);
  for (int64_t k = 0; k < n; ++k) out[k] = rng_u01(&g);
}

/* seeded Fisher-Yates permutation of 0..n-1 */
void wl_permutation(uint64_t seed, uint64_t stream, int64_t n, int64_t *perm) {
  wl_rng g;
  rng_seed(&g, seed, stream);
  for (int64_t k = 0; k < n; ++k) perm[k] = k;
  for (int64_t k = n - 1; k > 0; --k) {
    int64_t j = (int64_t)(rng_u01(&g) * (double)(k + 1));
    if (j > k) j = k;
    int64_t t = perm[k];
    perm[k] = perm[j];
    perm[j] = t;
  }
}

static inline int wrapi(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

static inline double min_image(double d, double len) {
  if (d > 0.5 * len) return d - len;
  if (d < -0.5 * len) return d + len;
  return d;
}

/* counter-based uniform for trial positions: (seed, particle, attempt, axis) -> [0,1) */
static inline double trial_u01(uint64_t seed, int64_t i, int64_t a, int k) {
  uint64_t x = seed ^ ((uint64_t)i * 0xD1B54A32D192ED03ULL) ^ ((uint64_t)a * 0xAEF17502108EF2D9ULL) ^
               ((uint64_t)k * 0x9E3779B97F4A7C15ULL);
  (void)splitmix64(&x);
  uint64_t z = splitmix64(&x);
  return (double)(z >> 11) * 0x1.0p-53;
}

typedef struct {
  int nc[3];
  double h[3], len[3];
  int cap;
  int32_t *cnt;
  double *cell; /* per cell: cap entries of (x, y, z, r) */
} rsa_grid;

static inline int64_t grid_cell(const rsa_grid *G, const double p[3], int c[3]) {
  for (int a = 0; a < 3; ++a) {
    c[a] = (int)(p[a] / G->h[a]);
    if (c[a] >= G->nc[a]) c[a] = G->nc[a] - 1;
  }
  return ((int64_t)c[2] * G->nc[1] + c[1]) * G->nc[0] + c[0];
}

/* 1 if sphere (p, ri) overlaps nothing stored in the grid */
static int grid_free(const rsa_grid *G, const double p[3], double ri) {
  int c[3];
  (void)grid_cell(G, p, c);
  const int lo0 = G->nc[0] == 1 ? 0 : -1, hi0 = G->nc[0] == 1 ? 0 : 1;
  const int lo1 = G->nc[1] == 1 ? 0 : -1, hi1 = G->nc[1] == 1 ? 0 : 1;
  const int lo2 = G->nc[2] == 1 ? 0 : -1, hi2 = G->nc[2] == 1 ? 0 : 1;
  for (int dz = lo2; dz <= hi2; ++dz) {
    const int cz = wrapi(c[2] + dz, G->nc[2]);
    for (int dy = lo1; dy <= hi1; ++dy) {
      const int cy = wrapi(c[1] + dy, G->nc[1]);
      for (int dx = lo0; dx <= hi0; ++dx) {
        const int cx = wrapi(c[0] + dx, G->nc[0]);
        const int64_t cid = ((int64_t)cz * G->nc[1] + cy) * G->nc[0] + cx;
        const double *q = G->cell + (size_t)cid * G->cap * 4;
        const int m = G->cnt[cid];
        for (int k = 0; k < m; ++k, q += 4) {
          const double d0 = min_image(q[0] - p[0], G->len[0]);
          const double d1 = min_image(q[1] - p[1], G->len[1]);
          const double d2 = min_image(q[2] - p[2], G->len[2]);
          const double s = q[3] + ri;
          if (d0 * d0 + d1 * d1 + d2 * d2 <= s * s) return 0;
        }
      }
    }
  }
  return 1;
}

/*
 * RSA placement of n spheres with radii r[] into the periodic box
 * [0,len0) x [0,len1) x [0,len2).  Writes x, y, z.
 *
 * Trials run in batches of up to B = clamp(n/256, 1, 8192) pending spheres,
 * oldest first: every batch
 * member draws one trial point (a counter-based draw from (seed, sphere,
 * attempt)), all are tested in parallel against the spheres already placed,
 * and the survivors are then accepted in batch order unless they overlap a
 * sphere accepted earlier in the same batch.  Rejected spheres stay at the
 * head of the queue.  The result does not depend on the thread count.
 *
 * Returns the total number of trials, or a negative code:
 *   -1 a sphere could not be placed within max_trials trials,
 *   -2 out of memory, -3 a grid cell overflowed its capacity (retry larger cap).
 */
int64_t wl_rsa(uint64_t seed, int64_t n, const double *r, double len0, double len1, double len2,
               int64_t max_trials, int cap, double *x, double *y, double *z) {
  if (n <= 0) return 0;
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) rmax = r[i] > rmax ? r[i] : rmax;
  rsa_grid G;
  G.len[0] = len0;
  G.len[1] = len1;
  G.len[2] = len2;
  G.cap = cap;
  for (int a = 0; a < 3; ++a) {
    G.nc[a] = (int)floor(G.len[a] / (2.0 * rmax * (1.0 + 1e-9)));
    if (G.nc[a] < 3) G.nc[a] = 1; /* tiny axis: one cell, minimum image only */
    if (G.nc[a] > 4096) G.nc[a] = 4096;
    G.h[a] = G.len[a] / G.nc[a];
  }
  const int64_t ncell = (int64_t)G.nc[0] * G.nc[1] * G.nc[2];
  /* batch size bounded by n/256 so that no sphere is overtaken by more than
   * n/256 later ones: the order of placement stays close to the given order */
  int64_t B = n / 256;
  if (B < 1) B = 1;
  if (B > 8192) B = 8192;
  G.cnt = (int32_t *)calloc((size_t)ncell, sizeof(int32_t));
  G.cell = (double *)malloc((size_t)ncell * (size_t)cap * 4 * sizeof(double));
  int64_t *queue = (int64_t *)malloc((size_t)B * sizeof(int64_t));
  int64_t *attempts = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  double *cand = (double *)malloc((size_t)B * 3 * sizeof(double));
  unsigned char *ok = (unsigned char *)malloc((size_t)B);
  /* per-batch spatial hash of accepted trial points: cell id -> chain */
  const int64_t HS = 4 * B;
  int64_t *hkey = (int64_t *)malloc((size_t)HS * sizeof(int64_t));
  int32_t *hhead = (int32_t *)malloc((size_t)HS * sizeof(int32_t));
  int32_t *hnext = (int32_t *)malloc((size_t)B * sizeof(int32_t));
  int64_t rc = 0;
  if (!G.cnt || !G.cell || !queue || !attempts || !cand || !ok || !hkey || !hhead || !hnext) {
    rc = -2;
    goto done;
  }
  int64_t nq = 0, next = 0, placed = 0, trials = 0;
  while (placed < n) {
    while (nq < B && next < n) queue[nq++] = next++;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nq; ++k) {
      const int64_t i = queue[k];
      double *p = cand + 3 * k;
      const double len[3] = {len0, len1, len2};
      for (int a = 0; a < 3; ++a) {
        p[a] = trial_u01(seed, i, attempts[i], a) * len[a];
        if (p[a] >= len[a]) p[a] = 0.0;
      }
      ok[k] = (unsigned char)grid_free(&G, p, r[i]);
    }
    trials += nq;
    for (int64_t s = 0; s < HS; ++s) hkey[s] = -1;
    int64_t keep = 0;
    for (int64_t k = 0; k < nq; ++k) {
      const int64_t i = queue[k];
      const double *p = cand + 3 * k;
      int c[3];
      const int64_t cid = grid_cell(&G, p, c);
      if (ok[k]) {
        /* conflicts with spheres accepted earlier in this batch */
        for (int dz = -1; dz <= 1 && ok[k]; ++dz)
          for (int dy = -1; dy <= 1 && ok[k]; ++dy)
            for (int dx = -1; dx <= 1 && ok[k]; ++dx) {
              const int64_t nb = ((int64_t)wrapi(c[2] + dz, G.nc[2]) * G.nc[1] + wrapi(c[1] + dy, G.nc[1])) *
                                     G.nc[0] + wrapi(c[0] + dx, G.nc[0]);
              int64_t slot = (int64_t)((uint64_t)nb * 0x9E3779B97F4A7C15ULL >> 20) % HS;
              while (hkey[slot] != -1 && hkey[slot] != nb) slot = (slot + 1) % HS;
              if (hkey[slot] != nb) continue;
              for (int32_t e = hhead[slot]; e >= 0; e = hnext[e]) {
                const double *q = cand + 3 * e;
                const double d0 = min_image(q[0] - p[0], len0);
                const double d1 = min_image(q[1] - p[1], len1);
                const double d2 = min_image(q[2] - p[2], len2);
                const double sr = r[queue[e]] + r[i];
                if (d0 * d0 + d1 * d1 + d2 * d2 <= sr * sr) {
                  ok[k] = 0;
                  break;
                }
              }
            }
      }
      if (ok[k]) {
        int64_t slot = (int64_t)((uint64_t)cid * 0x9E3779B97F4A7C15ULL >> 20) % HS;
        while (hkey[slot] != -1 && hkey[slot] != cid) slot = (slot + 1) % HS;
        if (hkey[slot] != cid) {
          hkey[slot] = cid;
          hhead[slot] = -1;
        }
        hnext[k] = hhead[slot];
        hhead[slot] = (int32_t)k;
        if (G.cnt[cid] >= cap) {
          rc = -3;
          goto done;
        }
        double *q = G.cell + ((size_t)cid * cap + (size_t)G.cnt[cid]) * 4;
        q[0] = p[0];
        q[1] = p[1];
        q[2] = p[2];
        q[3] = r[i];
        G.cnt[cid] += 1;
        x[i] = p[0];
        y[i] = p[1];
        z[i] = p[2];
        ++placed;
      } else {
        if (++attempts[i] >= max_trials) {
          rc = -1;
          goto done;
        }
      }
    }
    /* compact: rejected spheres keep their order at the head of the queue */
    for (int64_t k = 0; k < nq; ++k)
      if (!ok[k]) queue[keep++] = queue[k];
    nq = keep;
  }
  rc = trials;
done:
  free(G.cnt);
  free(G.cell);
  free(queue);
  free(attempts);
  free(cand);
  free(ok);
  free(hkey);
  free(hhead);
  free(hnext);
  return rc;
}
