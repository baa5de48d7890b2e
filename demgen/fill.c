/*
 * Epsilon priority-flood depression filling for synthetic DEM generation.
 *
 * Input generation only: this file computes no flow directions and no up-slope
 * area.  It makes a DEM satisfy the precondition of the paper (Sec. 3, first
 * paragraph: pits and flats removed beforehand) by the epsilon variant of the
 * Priority-Flood algorithm (Barnes, Lehman & Mulla 2014, "Priority-Flood: An
 * Optimal Depression-Filling and Watershed-Labeling Algorithm for Digital
 * Elevation Models"): seeds are the edge cells; cells are visited in increasing
 * elevation from a min-heap; a visited neighbour that is not strictly higher
 * than the cell that discovered it is raised to fl32(z + eps) and put on a FIFO
 * "pit" queue that is drained before the heap.  Every non-seed cell is therefore
 * strictly higher than the neighbour that discovered it.
 *
 * Edge (seed) cells: valid cells on the DEM boundary or 8-adjacent to a NaN
 * (NoData) cell.  NaN cells are never visited and stay NaN.
 *
 * Heap keys are (monotone float bits << 32 | cell index), so ties resolve by
 * cell index and the result is deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint32_t fkey(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

typedef struct { uint64_t* a; size_t n, cap; } heap_t;

static int heap_push(heap_t* h, uint64_t k) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? h->cap * 2 : 1024;
    uint64_t* na = (uint64_t*)realloc(h->a, nc * sizeof(uint64_t));
    if (!na) return -1;
    h->a = na; h->cap = nc;
  }
  size_t i = h->n++;
  while (i > 0) {
    size_t p = (i - 1) >> 1;
    if (h->a[p] <= k) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i] = k;
  return 0;
}

static uint64_t heap_pop(heap_t* h) {
  uint64_t top = h->a[0];
  uint64_t last = h->a[--h->n];
  size_t i = 0, n = h->n;
  for (;;) {
    size_t l = 2 * i + 1;
    if (l >= n) break;
    size_t m = (l + 1 < n && h->a[l + 1] < h->a[l]) ? l + 1 : l;
    if (h->a[m] >= last) break;
    h->a[i] = h->a[m];
    i = m;
  }
  if (n) h->a[i] = last;
  return top;
}

/* Returns 0 on success, -1 on allocation failure. */
int demgen_fill_eps(float* z, int64_t H, int64_t W, float eps) {
  static const int DR[8] = {0, -1, -1, -1, 0, 1, 1, 1};
  static const int DC[8] = {1, 1, 0, -1, -1, -1, 0, 1};
  const int64_t N = H * W;
  uint8_t* seen = (uint8_t*)calloc((size_t)N, 1);
  uint32_t* pit = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  heap_t h = {0, 0, 0};
  if (!seen || !pit) { free(seen); free(pit); return -1; }
  for (int64_t r = 0; r < H; ++r) {
    for (int64_t c = 0; c < W; ++c) {
      int64_t i = r * W + c;
      if (isnan(z[i])) continue;
      int edge = (r == 0 || c == 0 || r == H - 1 || c == W - 1);
      for (int d = 0; d < 8 && !edge; ++d) {
        if (isnan(z[(r + DR[d]) * W + c + DC[d]])) edge = 1;
      }
      if (edge) {
        seen[i] = 1;
        if (heap_push(&h, ((uint64_t)fkey(z[i]) << 32) | (uint64_t)i)) goto oom;
      }
    }
  }
  {
    size_t ph = 0, pt = 0; /* FIFO head/tail into pit[] (each cell enters once) */
    while (ph < pt || h.n) {
      uint32_t c;
      if (ph < pt) c = pit[ph++];
      else c = (uint32_t)(heap_pop(&h) & 0xffffffffu);
      int64_t r = c / W, col = c % W;
      float zc = z[c];
      for (int d = 0; d < 8; ++d) {
        int64_t rr = r + DR[d], cc = col + DC[d];
        if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
        int64_t n = rr * W + cc;
        if (seen[n] || isnan(z[n])) continue;
        seen[n] = 1;
        if (z[n] <= zc) {
          float up = zc + eps;
          if (!(up > zc)) up = nextafterf(zc, INFINITY);
          z[n] = up;
          pit[pt++] = (uint32_t)n;
        } else {
          if (heap_push(&h, ((uint64_t)fkey(z[n]) << 32) | (uint64_t)n)) goto oom;
        }
      }
    }
  }
  free(seen); free(pit); free(h.a);
  return 0;
oom:
  free(seen); free(pit); free(h.a);
  return -1;
}
