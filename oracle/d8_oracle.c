/*
 * CPU ORACLE for D8 flow directions and D8 up-slope area -- TEST INFRASTRUCTURE.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * this library.  The product path (the HIP library and its Python binding)
 * never links, imports or calls it, and shares no code, header or table with
 * it.
 *
 * Plain, single-threaded, obviously correct.  Floating-point sums are in fp64.
 * Method: Barnes, Lehman & Mulla, "Distributed Parallel D8 Up-Slope Area
 * Calculation in Digital Elevation Models", PDPTA 2011.
 *
 *   - Sec. 2, Eq. (1): A(p) = 1 + sum of A(i) over the neighbours i that drain
 *     into p.  Sec. 2 also allows per-cell weights, so A(p) = w(p) + sum A(i).
 *   - Sec. 1 (the D8 function of O'Callaghan & Mark): each cell sends all of its
 *     flow to the lowest of its eight neighbours; flows join but never split,
 *     so the flow graph is a forest.
 *   - Sec. 3, Alg. 1 (dependency counting) and Alg. 2 (queue-driven internal
 *     up-slope area) evaluate Eq. (1) in dependency order; here they run on the
 *     whole DEM as one partition with a plain FIFO queue (Kahn's order).
 *
 * Readings where the paper is silent:
 *   - "lowest" neighbour, strict '<', scanned in the order E,NE,N,NW,W,SW,S,SE;
 *     the first minimum wins; no strictly lower neighbour -> outlet (code 8).
 *   - row 0 is north; E = (r, c+1), N = (r-1, c).
 *   - every valid DEM-boundary cell, and every valid cell 8-adjacent to NoData
 *     (NaN), is an outlet (code 8); NaN cells get code 255 and area 0.
 *
 * Direction codes: 0 E, 1 NE, 2 N, 3 NW, 4 W, 5 SW, 6 S, 7 SE, 8 outlet,
 * 255 NoData.
 *
 * Parity status: flowdirs, accumulation (u32 and f64), backward and brute force
 * are pinned by tests that do not reuse this code (plane closed forms, the
 * serpentine closed forms, pure-Python brute force on tiny grids, a hand-worked
 * fixture, the recursion identity, the outlet-sum invariant, linearity and the
 * adjoint dot-product identity).
 */
#define _GNU_SOURCE /* M_SQRT1_2 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Oracle status values (independent of the product's status enum). */
#define ORC_OK 0
#define ORC_BADDIR 4 /* code not in {0..8, 255}, or a target off-grid / into NoData */
#define ORC_CYCLE 5  /* the direction field is not a forest */
#define ORC_NOMEM 2

static const int ODR[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int ODC[8] = {1, 1, 0, -1, -1, -1, 0, 1};

/* D8 "lowest of eight" direction field (Sec. 1; tie and edge readings above). */
int orc_flowdirs(const float* z, int64_t H, int64_t W, uint8_t* dirs) {
  for (int64_t r = 0; r < H; ++r) {
    for (int64_t c = 0; c < W; ++c) {
      int64_t i = r * W + c;
      float v = z[i];
      if (isnan(v)) { dirs[i] = 255; continue; }
      if (r == 0 || c == 0 || r == H - 1 || c == W - 1) { dirs[i] = 8; continue; }
      int nan_adj = 0;
      for (int d = 0; d < 8; ++d)
        if (isnan(z[(r + ODR[d]) * W + c + ODC[d]])) nan_adj = 1;
      if (nan_adj) { dirs[i] = 8; continue; }
      float best = v;
      int k = 8;
      for (int d = 0; d < 8; ++d) {
        float n = z[(r + ODR[d]) * W + c + ODC[d]];
        if (n < best) { best = n; k = d; }
      }
      dirs[i] = (uint8_t)k;
    }
  }
  return ORC_OK;
}

/* D8 steepest-slope direction field: the slope rule with diagonal distance of
 * Sec. 3 (drop divided by the distance to the neighbour: 1 for E, N, W, S and
 * sqrt(2) for the diagonals).  The slope of neighbour d is evaluated in double
 * as (z_c - z_d) * f_d with f_d = 1 or 1/sqrt(2) (rounded to double); the
 * largest strictly positive slope wins, ties to the first in E..SE order; no
 * positive slope -> outlet (8).  Edge and NoData rules as orc_flowdirs. */
int orc_flowdirs_steepest(const float* z, int64_t H, int64_t W, uint8_t* dirs) {
  for (int64_t r = 0; r < H; ++r) {
    for (int64_t c = 0; c < W; ++c) {
      int64_t i = r * W + c;
      float v = z[i];
      if (isnan(v)) { dirs[i] = 255; continue; }
      if (r == 0 || c == 0 || r == H - 1 || c == W - 1) { dirs[i] = 8; continue; }
      int nan_adj = 0;
      for (int d = 0; d < 8; ++d)
        if (isnan(z[(r + ODR[d]) * W + c + ODC[d]])) nan_adj = 1;
      if (nan_adj) { dirs[i] = 8; continue; }
      double best = 0.0;
      int k = 8;
      for (int d = 0; d < 8; ++d) {
        double n = (double)z[(r + ODR[d]) * W + c + ODC[d]];
        double f = (ODR[d] != 0 && ODC[d] != 0) ? M_SQRT1_2 : 1.0;
        double s = ((double)v - n) * f;
        if (s > best) { best = s; k = d; }
      }
      dirs[i] = (uint8_t)k;
    }
  }
  return ORC_OK;
}

/* Target of cell i, or -1 for an outlet / NoData; -2 for an invalid field. */
static int64_t target_of(const uint8_t* dirs, int64_t H, int64_t W, int64_t i) {
  uint8_t k = dirs[i];
  if (k == 8 || k == 255) return -1;
  if (k > 8) return -2;
  int64_t r = i / W + ODR[k], c = i % W + ODC[k];
  if (r < 0 || r >= H || c < 0 || c >= W) return -2;
  int64_t t = r * W + c;
  if (dirs[t] == 255) return -2;
  return t;
}

/* Checks the field; fills tgt[] (int64 per cell, -1 = none) and indeg[].
 * indeg counts the cells that drain into each cell (Alg. 1's dependency count). */
static int prepare(const uint8_t* dirs, int64_t H, int64_t W, int64_t* tgt, uint8_t* indeg,
                   int64_t* nvalid) {
  const int64_t N = H * W;
  int64_t nv = 0;
  memset(indeg, 0, (size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    int64_t t = target_of(dirs, H, W, i);
    if (t == -2) return ORC_BADDIR;
    tgt[i] = t;
    if (dirs[i] != 255) ++nv;
    if (t >= 0) indeg[t]++;
  }
  *nvalid = nv;
  return ORC_OK;
}

/* Kahn order of all valid cells (upstream before downstream); returns status. */
static int kahn_order(const uint8_t* dirs, int64_t N, const int64_t* tgt, uint8_t* indeg,
                      int64_t nvalid, uint32_t* order) {
  int64_t head = 0, tail = 0;
  for (int64_t i = 0; i < N; ++i)
    if (dirs[i] != 255 && indeg[i] == 0) order[tail++] = (uint32_t)i;
  while (head < tail) {
    uint32_t u = order[head++];
    int64_t t = tgt[u];
    if (t >= 0 && --indeg[t] == 0) order[tail++] = (uint32_t)t;
  }
  return tail == nvalid ? ORC_OK : ORC_CYCLE;
}

/* Eq. (1) with unit weights, uint32 counts, Alg. 1 + Alg. 2 with a FIFO queue. */
int orc_accum_u32(const uint8_t* dirs, int64_t H, int64_t W, uint32_t* A) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  uint32_t* q = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  int64_t* tgt = NULL;
  int st = ORC_NOMEM;
  int64_t nvalid = 0;
  /* targets are recomputed on the fly to keep memory at ~10 B/cell */
  if (!indeg || !q) goto out;
  memset(indeg, 0, (size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    int64_t t = target_of(dirs, H, W, i);
    if (t == -2) { st = ORC_BADDIR; goto out; }
    if (dirs[i] != 255) ++nvalid;
    if (t >= 0) indeg[t]++;
    A[i] = dirs[i] == 255 ? 0u : 1u;
  }
  {
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < N; ++i)
      if (dirs[i] != 255 && indeg[i] == 0) q[tail++] = (uint32_t)i;
    while (head < tail) {
      uint32_t u = q[head++];
      int64_t t = target_of(dirs, H, W, u);
      if (t >= 0) {
        A[t] += A[u];
        if (--indeg[t] == 0) q[tail++] = (uint32_t)t;
      }
    }
    st = (tail == nvalid) ? ORC_OK : ORC_CYCLE;
  }
out:
  free(indeg); free(q); free(tgt);
  return st;
}

/* Eq. (1) with weights w (float32 in, NULL = unit), fp64 sums. */
int orc_accum_f64(const uint8_t* dirs, int64_t H, int64_t W, const float* w, double* A) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  int64_t* tgt = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  uint32_t* order = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  int st = ORC_NOMEM;
  int64_t nvalid = 0;
  if (!indeg || !tgt || !order) goto out;
  st = prepare(dirs, H, W, tgt, indeg, &nvalid);
  if (st != ORC_OK) goto out;
  for (int64_t i = 0; i < N; ++i) A[i] = dirs[i] == 255 ? 0.0 : (w ? (double)w[i] : 1.0);
  st = kahn_order(dirs, N, tgt, indeg, nvalid, order);
  if (st != ORC_OK) goto out;
  for (int64_t j = 0; j < nvalid; ++j) {
    uint32_t u = order[j];
    if (tgt[u] >= 0) A[tgt[u]] += A[u];
  }
out:
  free(indeg); free(tgt); free(order);
  return st;
}

/* Adjoint of the weighted accumulation: A = (I - P)^-1 w, so the gradient of a
 * loss with respect to w is (I - P)^-T g, i.e. G(c) = g(c) + G(target(c)):
 * the sum of g along c's downstream path, c included.  Evaluated in reverse
 * Kahn order (downstream before upstream).  g is float32 (NULL = unit). */
int orc_backward_f64(const uint8_t* dirs, int64_t H, int64_t W, const float* g, double* G) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  int64_t* tgt = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  uint32_t* order = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  int st = ORC_NOMEM;
  int64_t nvalid = 0;
  if (!indeg || !tgt || !order) goto out;
  st = prepare(dirs, H, W, tgt, indeg, &nvalid);
  if (st != ORC_OK) goto out;
  st = kahn_order(dirs, N, tgt, indeg, nvalid, order);
  if (st != ORC_OK) goto out;
  for (int64_t i = 0; i < N; ++i) G[i] = dirs[i] == 255 ? 0.0 : (g ? (double)g[i] : 1.0);
  for (int64_t j = nvalid - 1; j >= 0; --j) {
    uint32_t u = order[j];
    if (tgt[u] >= 0) G[u] += G[tgt[u]];
  }
out:
  free(indeg); free(tgt); free(order);
  return st;
}

/* Same as orc_backward_f64 but with fp64 upstream gradients. */
int orc_backward_f64d(const uint8_t* dirs, int64_t H, int64_t W, const double* g, double* G) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  int64_t* tgt = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  uint32_t* order = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  int st = ORC_NOMEM;
  int64_t nvalid = 0;
  if (!indeg || !tgt || !order) goto out;
  st = prepare(dirs, H, W, tgt, indeg, &nvalid);
  if (st != ORC_OK) goto out;
  st = kahn_order(dirs, N, tgt, indeg, nvalid, order);
  if (st != ORC_OK) goto out;
  for (int64_t i = 0; i < N; ++i) G[i] = dirs[i] == 255 ? 0.0 : g[i];
  for (int64_t j = nvalid - 1; j >= 0; --j) {
    uint32_t u = order[j];
    if (tgt[u] >= 0) G[u] += G[tgt[u]];
  }
out:
  free(indeg); free(tgt); free(order);
  return st;
}

/* Same as orc_accum_f64 but with fp64 weights. */
int orc_accum_f64d(const uint8_t* dirs, int64_t H, int64_t W, const double* w, double* A) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  int64_t* tgt = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  uint32_t* order = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  int st = ORC_NOMEM;
  int64_t nvalid = 0;
  if (!indeg || !tgt || !order) goto out;
  st = prepare(dirs, H, W, tgt, indeg, &nvalid);
  if (st != ORC_OK) goto out;
  for (int64_t i = 0; i < N; ++i) A[i] = dirs[i] == 255 ? 0.0 : w[i];
  st = kahn_order(dirs, N, tgt, indeg, nvalid, order);
  if (st != ORC_OK) goto out;
  for (int64_t j = 0; j < nvalid; ++j) {
    uint32_t u = order[j];
    if (tgt[u] >= 0) A[tgt[u]] += A[u];
  }
out:
  free(indeg); free(tgt); free(order);
  return st;
}

/* Brute force straight from the physical definition in Sec. 2: every valid cell
 * s adds its weight to every cell its flow passes through, s included.
 * O(N * path length); tiny grids only.  Guard: a path longer than N cells means
 * a cycle. */
int orc_bruteforce_f64(const uint8_t* dirs, int64_t H, int64_t W, const float* w, double* A) {
  const int64_t N = H * W;
  for (int64_t i = 0; i < N; ++i) A[i] = 0.0;
  for (int64_t s = 0; s < N; ++s) {
    if (dirs[s] == 255) continue;
    double ws = w ? (double)w[s] : 1.0;
    int64_t u = s, steps = 0;
    for (;;) {
      A[u] += ws;
      int64_t t = target_of(dirs, H, W, u);
      if (t == -2) return ORC_BADDIR;
      if (t < 0) break;
      if (++steps > N) return ORC_CYCLE;
      u = t;
    }
  }
  return ORC_OK;
}

/* Longest upstream dependency chain ending at each cell (cells, inclusive);
 * returns the maximum over the DEM, or -1 on error. */
int64_t orc_depth(const uint8_t* dirs, int64_t H, int64_t W) {
  const int64_t N = H * W;
  uint8_t* indeg = (uint8_t*)malloc((size_t)N);
  int64_t* tgt = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  uint32_t* order = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  uint32_t* d = (uint32_t*)calloc((size_t)N, sizeof(uint32_t));
  int64_t best = -1, nvalid = 0;
  if (!indeg || !tgt || !order || !d) goto out;
  if (prepare(dirs, H, W, tgt, indeg, &nvalid) != ORC_OK) goto out;
  if (kahn_order(dirs, N, tgt, indeg, nvalid, order) != ORC_OK) goto out;
  best = 0;
  for (int64_t j = 0; j < nvalid; ++j) {
    uint32_t u = order[j];
    d[u] += 1;
    if (d[u] > best) best = d[u];
    if (tgt[u] >= 0 && d[tgt[u]] < d[u]) d[tgt[u]] = d[u];
  }
out:
  free(indeg); free(tgt); free(order); free(d);
  return best;
}

/* ---------------------------------------------------------------------------
 * Depression and flat conditioning (Sec. 3, the preprocessing the method
 * assumes: pits raised to the level they drain at, flats given small
 * elevation changes).  The paper names no algorithm; the reading taken here is
 * the epsilon fill of Planchon & Darboux (2002):
 *
 *   seeds S = valid cells on the DEM boundary or 8-adjacent to NoData;
 *   inc(x) = fl32(x + eps) if that is > x, else the next float above x;
 *   F(s) = z(s) on S, and for every other valid cell
 *   F(c) = max(z(c), min over valid neighbours n of inc(F(n))).
 *
 * That fixed point is unique (inc is strictly increasing), F >= z, and every
 * non-seed cell has a neighbour lower than itself, so lowest-of-eight leaves
 * outlets only at seeds.  Equivalently F(c) is the minimum over 8-connected
 * paths c = p0, p1, ..., pk in S of max_i inc^i(z(p_i)).
 *
 * Computed here by Dijkstra's label-setting order on that path cost (a binary
 * heap keyed by the monotone bits of F, ties by cell index, stale entries
 * skipped): the cost through a settled cell u of a neighbour n is
 * max(z(n), inc(F(u))), which is non-decreasing in F(u) and never below it.
 * NaN cells stay NaN.  eps must be a positive normal float.  Minimum and
 * maximum are taken in the total order of the float bit patterns (the
 * order of the values, with -0 below +0), so signed zeros are resolved the
 * same way by any evaluation order.
 * ------------------------------------------------------------------------- */
static uint32_t orc_fbits_key(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

static float orc_inc(float x, float eps) {
  float y = x + eps;
  if (!(y > x)) y = nextafterf(x, INFINITY);
  return y;
}

typedef struct { uint64_t* a; size_t n, cap; } orc_heap;

static int orc_heap_push(orc_heap* h, uint64_t k) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? 2 * h->cap : 1024;
    uint64_t* na = (uint64_t*)realloc(h->a, nc * sizeof(uint64_t));
    if (!na) return -1;
    h->a = na;
    h->cap = nc;
  }
  size_t i = h->n++;
  while (i > 0) {
    size_t p = (i - 1) / 2;
    if (h->a[p] <= k) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i] = k;
  return 0;
}

static uint64_t orc_heap_pop(orc_heap* h) {
  uint64_t top = h->a[0], last = h->a[--h->n];
  size_t i = 0;
  for (;;) {
    size_t l = 2 * i + 1;
    if (l >= h->n) break;
    size_t m = (l + 1 < h->n && h->a[l + 1] < h->a[l]) ? l + 1 : l;
    if (h->a[m] >= last) break;
    h->a[i] = h->a[m];
    i = m;
  }
  if (h->n) h->a[i] = last;
  return top;
}

int orc_fill_eps(const float* z, int64_t H, int64_t W, float eps, float* F) {
  const int64_t N = H * W;
  if (N > 0xFFFFFFFFll) return ORC_NOMEM;
  uint8_t* done = (uint8_t*)calloc((size_t)(N ? N : 1), 1);
  orc_heap h = {0, 0, 0};
  int st = ORC_OK;
  if (!done) return ORC_NOMEM;
  for (int64_t r = 0; r < H; ++r) {
    for (int64_t c = 0; c < W; ++c) {
      const int64_t i = r * W + c;
      if (isnan(z[i])) { F[i] = z[i]; continue; }
      int seed = (r == 0 || c == 0 || r == H - 1 || c == W - 1);
      for (int d = 0; d < 8 && !seed; ++d)
        if (isnan(z[(r + ODR[d]) * W + c + ODC[d]])) seed = 1;
      F[i] = seed ? z[i] : INFINITY;
      if (seed && orc_heap_push(&h, ((uint64_t)orc_fbits_key(z[i]) << 32) | (uint64_t)i)) { st = ORC_NOMEM; goto out; }
    }
  }
  while (h.n) {
    const uint64_t k = orc_heap_pop(&h);
    const int64_t u = (int64_t)(k & 0xFFFFFFFFu);
    if (done[u] || (uint32_t)(k >> 32) != orc_fbits_key(F[u])) continue; /* stale */
    done[u] = 1;
    const int64_t r = u / W, c = u % W;
    const float through = orc_inc(F[u], eps);
    for (int d = 0; d < 8; ++d) {
      const int64_t rr = r + ODR[d], cc = c + ODC[d];
      if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
      const int64_t n = rr * W + cc;
      if (done[n] || isnan(z[n])) continue;
      /* max and < in the total order of the monotone bits (-0 below +0) */
      const float cand = orc_fbits_key(z[n]) > orc_fbits_key(through) ? z[n] : through;
      if (orc_fbits_key(cand) < orc_fbits_key(F[n])) {
        F[n] = cand;
        if (orc_heap_push(&h, ((uint64_t)orc_fbits_key(cand) << 32) | (uint64_t)n)) { st = ORC_NOMEM; goto out; }
      }
    }
  }
out:
  free(done);
  free(h.a);
  return st;
}
