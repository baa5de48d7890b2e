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
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static inline uint32_t fkey(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

/* Radix heap (Ahuja, Mehlhorn, Orlin & Tarjan 1990) over 64-bit keys.  Valid
 * because the flood is monotone: every key pushed after the first pop is
 * larger than the last key popped.  Keys are unique (the cell index is in the
 * low bits), so pops come out in exactly the order of a binary heap. */
typedef struct { uint64_t* a; size_t n, cap; } vec_t;
typedef struct { vec_t b[65]; uint64_t last; size_t n; } heap_t;

static int vec_push(vec_t* v, uint64_t k) {
  if (v->n == v->cap) {
    size_t nc = v->cap ? v->cap * 2 : 256;
    uint64_t* na = (uint64_t*)realloc(v->a, nc * sizeof(uint64_t));
    if (!na) return -1;
    v->a = na; v->cap = nc;
  }
  v->a[v->n++] = k;
  return 0;
}

static inline int bucket_of(uint64_t k, uint64_t last) {
  uint64_t x = k ^ last;
  return x ? 64 - __builtin_clzll(x) : 0;
}

static int heap_push(heap_t* h, uint64_t k) {
  h->n++;
  return vec_push(&h->b[bucket_of(k, h->last)], k);
}

static uint64_t heap_pop(heap_t* h) {
  if (h->b[0].n == 0) {
    int i = 1;
    while (h->b[i].n == 0) ++i;
    vec_t* v = &h->b[i];
    uint64_t m = v->a[0];
    for (size_t j = 1; j < v->n; ++j) if (v->a[j] < m) m = v->a[j];
    h->last = m;
    for (size_t j = 0; j < v->n; ++j) {
      /* every key of bucket i lands in a lower bucket; cannot fail to grow
         beyond what was already allocated in total, but check anyway */
      if (vec_push(&h->b[bucket_of(v->a[j], m)], v->a[j])) return ~(uint64_t)0;
    }
    v->n = 0;
  }
  h->n--;
  return h->b[0].a[--h->b[0].n];
}

static void heap_free(heap_t* h) {
  for (int i = 0; i < 65; ++i) free(h->b[i].a);
}

/* Returns 0 on success, -1 on allocation failure.  If progress > 0, a line
 * is written to stderr each time another `progress` cells have been settled. */
int demgen_fill_eps(float* z, int64_t H, int64_t W, float eps, int64_t progress) {
  static const int DR[8] = {0, -1, -1, -1, 0, 1, 1, 1};
  static const int DC[8] = {1, 1, 0, -1, -1, -1, 0, 1};
  const int64_t N = H * W;
  uint8_t* seen = (uint8_t*)calloc((size_t)N, 1);
  uint32_t* pit = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
  heap_t h;
  memset(&h, 0, sizeof(h));
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
    int64_t done = 0;
    while (ph < pt || h.n) {
      if (progress > 0 && ++done % progress == 0) {
        fprintf(stderr, "[demgen] fill: %lld of %lld cells settled\n", (long long)done, (long long)N);
        fflush(stderr);
      }
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
  free(seen); free(pit); heap_free(&h);
  return 0;
oom:
  free(seen); free(pit); heap_free(&h);
  return -1;
}
