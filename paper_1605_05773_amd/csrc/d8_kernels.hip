// gfx950 kernels of the D8 library: flow directions, tile passes and the
// perimeter-graph resolve.
//
// Scheme (Sec. 3 of Barnes, Lehman & Mulla, PDPTA 2011, on one GPU):
//   tile pass, emit   each TS x TS tile computes its internal up-slope area
//                     with the inflows from other tiles left out (Alg. 1-3),
//                     and writes, per perimeter cell, the partial area of
//                     every exit (a cell draining into another tile) and, for
//                     every receiver (a cell fed from another tile), the exit
//                     its in-tile path leaves by (Alg. 4's Cell_V / Origin).
//   resolve           exits form a forest (exit -> the exit reached from its
//                     target receiver); its subtree sums are the full areas of
//                     the exits (Alg. 5-6).  Computed in O(log depth) rounds.
//   tile pass, final  each tile recomputes its internal area with the resolved
//                     inflow of each receiver added, i.e. adds the incoming
//                     areas along the receivers' downstream paths (Alg. 7-8).
#include <algorithm>
#include <type_traits>

#include "d8_internal.hpp"
#include "d8.h"

namespace d8 {

// Optional per-phase cycle stamps for measurement builds (no-op here):
// D8_STAMP(pass, i) marks the start of phase i of pass 0 (emit), 1 (finalise),
// 2 (super-block up) or 3 (super-block down).
#ifndef D8_STAMP
#define D8_STAMP(pass, i)
#endif

constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr uint64_t kPendOne = 1ull << 40;

// ------------------------------------------------------------------ flowdirs --
// D8 "lowest of eight" (Sec. 1): a 16x8-thread block covers a 64x64-cell
// block; each thread owns 4 columns x 8 rows and reads its 10x6 neighbourhood.
constexpr int kFdTile = 64;
constexpr int kFdRows = 8;  // rows per thread (measured best of 4, 8, 16)

__device__ __forceinline__ uint8_t lowest8(float c, float n0, float n1, float n2, float n3, float n4, float n5,
                                           float n6, float n7) {
  // NaN neighbours never reach here (such cells are outlets).
  float best = c;
  uint8_t k = kNone;
  if (n0 < best) { best = n0; k = 0; }
  if (n1 < best) { best = n1; k = 1; }
  if (n2 < best) { best = n2; k = 2; }
  if (n3 < best) { best = n3; k = 3; }
  if (n4 < best) { best = n4; k = 4; }
  if (n5 < best) { best = n5; k = 5; }
  if (n6 < best) { best = n6; k = 6; }
  if (n7 < best) { best = n7; k = 7; }
  return k;
}

// Steepest-slope variant (the drop-over-distance rule of Sec. 3): slope to a
// neighbour = drop / distance, distance sqrt(2) for the diagonals, evaluated
// in double as (c - n) * f with f = 1 or 1/sqrt(2) rounded to double; the
// largest strictly positive slope wins, ties to the first in E..SE order.
__device__ __forceinline__ uint8_t steepest8(float c, float n0, float n1, float n2, float n3, float n4, float n5,
                                             float n6, float n7) {
  constexpr double kDiag = 0.70710678118654752440;
  const double z = (double)c;
  double best = 0.0;
  uint8_t k = kNone;
  double s;
  s = (z - (double)n0);         if (s > best) { best = s; k = 0; }
  s = (z - (double)n1) * kDiag; if (s > best) { best = s; k = 1; }
  s = (z - (double)n2);         if (s > best) { best = s; k = 2; }
  s = (z - (double)n3) * kDiag; if (s > best) { best = s; k = 3; }
  s = (z - (double)n4);         if (s > best) { best = s; k = 4; }
  s = (z - (double)n5) * kDiag; if (s > best) { best = s; k = 5; }
  s = (z - (double)n6);         if (s > best) { best = s; k = 6; }
  s = (z - (double)n7) * kDiag; if (s > best) { best = s; k = 7; }
  return k;
}

// A 16 x (64 / RPT) thread block covers a 64 x 64 block of cells; each thread
// owns 4 columns x RPT rows and reads its (RPT + 2) x 6 neighbourhood.
template <bool STEEP, int RPT>
__global__ __launch_bounds__(16 * (64 / RPT)) void k_flowdirs(const float* __restrict__ dem,
                                                             uint8_t* __restrict__ dirs, DemTable tab) {
  const int64_t tile = blockIdx.x;
  const DemInfo dm = dem_of_tile(tab, tile);
  const uint32_t lt = (uint32_t)(tile - dm.tile0);  // below 2^32: a 32-bit division
  const int64_t ty = lt / (uint32_t)dm.TX, tx = lt - (uint32_t)ty * (uint32_t)dm.TX;
  const int64_t H = dm.H, W = dm.W;
  const float* z = dem + dm.off;
  uint8_t* d = dirs + dm.off;
  const int64_t y0 = ty * kFdTile + RPT * threadIdx.y;
  const int64_t x0 = tx * kFdTile + 4 * threadIdx.x;
  if (y0 >= H || x0 >= W) return;
  float v[RPT + 2][6];
  // Threads whose neighbourhood lies inside the DEM read the middle four
  // columns of each row as one aligned 16-byte load.
  const bool vec = ((reinterpret_cast<uintptr_t>(z) & 15) == 0) && (W & 3) == 0 && y0 >= 1 && y0 + RPT < H &&
                   x0 >= 1 && x0 + 4 < W;
  if (vec) {
#pragma unroll
    for (int rr = 0; rr < RPT + 2; ++rr) {
      const float* row = z + (y0 - 1 + rr) * W + x0;
      const float4 q = *reinterpret_cast<const float4*>(row);
      v[rr][0] = row[-1];
      v[rr][1] = q.x;
      v[rr][2] = q.y;
      v[rr][3] = q.z;
      v[rr][4] = q.w;
      v[rr][5] = row[4];
    }
  } else {
#pragma unroll
    for (int rr = 0; rr < RPT + 2; ++rr) {
      const int64_t yy = y0 - 1 + rr;
      const bool rin = yy >= 0 && yy < H;
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) {
        const int64_t xx = x0 - 1 + cc;
        v[rr][cc] = (rin && xx >= 0 && xx < W) ? z[yy * W + xx] : 0.0f;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < RPT; ++a) {
    const int64_t y = y0 + a;
    if (y >= H) break;
    uint8_t code[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t x = x0 + b;
      const float c = v[a + 1][b + 1];
      uint8_t k;
      if (__builtin_isnan(c)) {
        k = kNoData;
      } else if (y == 0 || x == 0 || y == H - 1 || x >= W - 1) {
        k = kNone;
      } else {
        const float n0 = v[a + 1][b + 2], n1 = v[a][b + 2], n2 = v[a][b + 1], n3 = v[a][b];
        const float n4 = v[a + 1][b], n5 = v[a + 2][b], n6 = v[a + 2][b + 1], n7 = v[a + 2][b + 2];
        const bool nanadj = __builtin_isnan(n0) | __builtin_isnan(n1) | __builtin_isnan(n2) |
                            __builtin_isnan(n3) | __builtin_isnan(n4) | __builtin_isnan(n5) |
                            __builtin_isnan(n6) | __builtin_isnan(n7);
        k = nanadj ? kNone
                   : (STEEP ? steepest8(c, n0, n1, n2, n3, n4, n5, n6, n7)
                            : lowest8(c, n0, n1, n2, n3, n4, n5, n6, n7));
      }
      code[b] = k;
    }
    uint8_t* row = d + y * W + x0;
    if (x0 + 3 < W && ((reinterpret_cast<uintptr_t>(row) & 3) == 0)) {
      *reinterpret_cast<uint32_t*>(row) =
          (uint32_t)code[0] | ((uint32_t)code[1] << 8) | ((uint32_t)code[2] << 16) | ((uint32_t)code[3] << 24);
    } else {
      for (int b = 0; b < 4 && x0 + b < W; ++b) row[b] = code[b];
    }
  }
}

// Stage a BW x BH block of direction codes with a one-cell halo into LDS
// (row stride BW + 2).  When the block's rows are 4-byte aligned (full-width
// block, width and offset multiples of 4) the BH + 2 rows are fetched as
// 32-bit words, all loads of a thread issued before any is consumed; the two
// halo columns are single bytes.
// NTC is the workgroup size when known at compile time (0: blockDim.x).
template <int BW, int BH, int NTC = 0>
__device__ __forceinline__ void load_halo(uint8_t* code, const uint8_t* __restrict__ dirs, const DemInfo& dm,
                                          int64_t y0, int64_t x0, int bw) {
  constexpr int HS = BW + 2;
  constexpr int HR = BH + 2;
  constexpr int WPR = BW / 4;     // 32-bit words per block row
  constexpr int NW = HR * WPR;    // rows y0-1 .. y0+BH
  constexpr int MAXW = NTC ? (NW + NTC - 1) / NTC : 9;
  constexpr int HL = NTC ? (2 * HR + NTC - 1) / NTC : 2;  // halo-column bytes per thread
  const uint8_t* D = dirs + dm.off;
  const int64_t H = dm.H, W = dm.W;
  const int NT = NTC ? NTC : (int)blockDim.x, tid = threadIdx.x;
  const bool vec = bw == BW && (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(D + x0) & 3) == 0) &&
                   (NW + NT - 1) / NT <= MAXW && 2 * HR <= HL * NT;
  if (vec) {
    uint32_t v[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
      const int i = tid + k * NT;
      v[k] = 0xFEFEFEFEu;  // kOutside bytes
      if (i < NW) {
        const int lr = i / WPR, q = i - lr * WPR;
        const int64_t gy = y0 + lr - 1;
        if (gy >= 0 && gy < H) v[k] = *reinterpret_cast<const uint32_t*>(D + gy * W + x0 + 4 * q);
      }
    }
    // halo columns x0-1 and x0+BW (2*HR bytes; at most HL per thread)
    uint8_t hb[HL];
    int hidx[HL];
#pragma unroll
    for (int k = 0; k < HL; ++k) {
      hb[k] = kOutside;
      hidx[k] = -1;
      const int i = tid + k * NT;
      if (i < 2 * HR) {
        const int lr = i >> 1, side = i & 1;
        const int64_t gy = y0 + lr - 1, gx = side ? x0 + BW : x0 - 1;
        hidx[k] = lr * HS + (side ? HS - 1 : 0);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) hb[k] = D[gy * W + gx];
      }
    }
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
      const int i = tid + k * NT;
      if (i < NW) {
        const int lr = i / WPR, q = i - lr * WPR;
        uint8_t* o = code + lr * HS + 1 + 4 * q;
        o[0] = (uint8_t)v[k];
        o[1] = (uint8_t)(v[k] >> 8);
        o[2] = (uint8_t)(v[k] >> 16);
        o[3] = (uint8_t)(v[k] >> 24);
      }
    }
#pragma unroll
    for (int k = 0; k < HL; ++k)
      if (hidx[k] >= 0) code[hidx[k]] = hb[k];
  } else {
    for (int i = tid; i < HS * HR; i += NT) {
      const int lr = i / HS, lc = i - lr * HS;
      const int64_t gy = y0 + lr - 1, gx = x0 + lc - 1;
      uint8_t v = kOutside;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = D[gy * W + gx];
      code[i] = v;
    }
  }
}

// Masks of the inputs of in-tile cell (r, c): bit i set if the neighbour at
// offset i drains into the cell; split into inputs inside the tile and inputs
// from outside it (receivers).  Branch-free.
template <int TS>
__device__ __forceinline__ uint32_t input_mask(const uint8_t* code, int r, int c) {
  constexpr int HS = TS + 2;
  const uint8_t* p = code + (r + 1) * HS + c + 1;
  uint32_t m = 0;
  m |= (uint32_t)(p[1] == 4) << 0;        // E neighbour drains W
  m |= (uint32_t)(p[1 - HS] == 5) << 1;   // NE drains SW
  m |= (uint32_t)(p[-HS] == 6) << 2;      // N drains S
  m |= (uint32_t)(p[-1 - HS] == 7) << 3;  // NW drains SE
  m |= (uint32_t)(p[-1] == 0) << 4;       // W drains E
  m |= (uint32_t)(p[HS - 1] == 1) << 5;   // SW drains NE
  m |= (uint32_t)(p[HS] == 2) << 6;       // S drains N
  m |= (uint32_t)(p[HS + 1] == 3) << 7;   // SE drains NW
  return m;
}

// Directions i whose neighbour (r + ddr(i), c + ddc(i)) lies outside the tile.
__device__ __forceinline__ uint32_t outside_dirs(int r, int c, int tw, int th) {
  const uint32_t n = r == 0 ? 0x0Eu : 0u;        // NE N NW
  const uint32_t s = r == th - 1 ? 0xE0u : 0u;   // SW S SE
  const uint32_t w = c == 0 ? 0x38u : 0u;        // NW W SW
  const uint32_t e = c == tw - 1 ? 0x83u : 0u;   // E NE SE
  return n | s | w | e;
}

template <int TS>
__device__ __forceinline__ void inputs_of(const uint8_t* code, int r, int c, const TileGeo& g, int& pend,
                                          uint32_t& inm, uint32_t& ext) {
  const uint32_t m = input_mask<TS>(code, r, c);
  const uint32_t out = outside_dirs(r, c, g.tw, g.th);
  inm = m & ~out;
  ext = m & out;
  pend = __builtin_popcount(inm);
}

template <int TS>
__device__ __forceinline__ uint32_t ext_mask(const uint8_t* code, int r, int c, const TileGeo& g) {
  return input_mask<TS>(code, r, c) & outside_dirs(r, c, g.tw, g.th);
}

// Sum of the resolved areas of the exits (in other tiles) that drain into
// receiver (r, c): the inflow the paper's master returns for a receiver.
// A cell has at most 5 outside neighbours (a tile corner); all loads are
// issued before the first is used.
template <typename V>
__device__ __forceinline__ V gather_inflow(const V* __restrict__ F, uint32_t ext, int r, int c, const TileGeo& g,
                                           int ts, int cap) {
  int64_t sl[5];
  uint32_t m = ext;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const uint32_t i = m ? (uint32_t)__builtin_ctz(m) : 0u;
    const int64_t gy = g.y0 + r + ddr(i), gx = g.x0 + c + ddc(i);
    sl[k] = m ? slot_of_cell(g.dm, gy, gx, ts, cap) : -1;
    m &= m - 1;
  }
  V t[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) t[k] = F[sl[k] >= 0 ? sl[k] : 0];
  V x = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) x += sl[k] >= 0 ? t[k] : (V)0;
  return x;
}

// Lanes of a wave that add to the same LDS address in one instruction
// serialise.  For a pair of adjacent lanes adding to the same target, the
// right lane (`right`; never lane 0 of the wave) hands its value to the left
// one by DPP and skips its add; returns true for such a right lane.  Lanes
// with `valid` false add nothing.  Every lane of the wave must call it.  The
// shifts write 0 where the source lane is beyond the wave (bound_ctrl), so
// lane 63, which has no right neighbour, gains 0.
template <typename V>
__device__ __forceinline__ bool merge_pair_add(uint32_t target, bool valid, bool right, V& v) {
  const uint32_t tl = (uint32_t)__builtin_amdgcn_mov_dpp((int)target, 0x138, 0xF, 0xF, true);  // lane - 1 (wave_shr:1)
  const bool dup = right & valid & (tl == target);
  const V give = dup ? v : (V)0;
  V gain;
  if constexpr (sizeof(V) == 4) {
    gain = __builtin_bit_cast(V, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, give), 0x130, 0xF, 0xF, true));
  } else {
    const uint64_t gb = __builtin_bit_cast(uint64_t, give);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)gb, 0x130, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(gb >> 32), 0x130, 0xF, 0xF, true);
    gain = __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);  // lane + 1 (wave_shl:1)
  }
  if (valid) v += gain;
  return dup;
}

// Termination flags of the doubling loops: two LDS words used alternately,
// so each round needs only its two barriers (a reduction barrier would add
// two more).  Round j sets flag[j & 1] after the middle barrier; thread 0
// clears flag[(j + 1) & 1], which every thread finished reading before that
// barrier.
struct RoundFlag {
  uint32_t f[2];
};

// --------------------------------------------------- counts: tile doubling --
// A workgroup owns a BW x BH block of cells made of whole TS x TS tiles (the
// tiles of a block are independent).  Inside a tile the up-slope area with
// unknown inflows (Alg. 2) is A = (I - P)^-1 w, evaluated as
// (I + P)(I + P^2)(I + P^4)... w: in round j every cell whose 2^j-th in-tile
// ancestor exists adds its current value to that ancestor, then jumps its
// ancestor pointer to the ancestor's ancestor.  After ceil(log2(depth)) rounds
// every cell holds its tile-local area.  Control flow is uniform and cells
// close to their tile root drop out early; integer sums make the result
// independent of the order of the atomic additions.
constexpr uint16_t kNoAnc = 0xFFFF;

// Per cell: value, and a link word (low 16 bits: the exact 2^j-th in-tile
// ancestor or kNoAnc; high 16 bits: the ancestor at distance
// min(2^j, distance to the tile root), i.e. the root once the exact
// ancestor has run out).  The tile pass keeps both halves as byte offsets
// into the link array (4 x the cell index: below 2^16 for blocks of up to
// 16384 cells, and never kNoAnc), so that a pointer is an LDS address.
template <int BW, int BH, typename V>
struct DblSmem {
  union {
    struct {
      V val[BW * BH];
      uint32_t link[BW * BH];
    };
    float z[(BW + 4) * (BH + 4)];  // fused call: the DEM block with a 2-cell halo
  };
  uint8_t code[(BW + 2) * (BH + 2)];
};

// Fused call: D8 codes of the block and its 1-cell halo computed from the DEM
// (same rule as k_flowdirs) into `code`; the block's own codes are written to
// `dirs` for the finalising pass.  Cells beyond the DEM get kOutside.
template <int BW, int BH, int NT, typename SM>
__device__ __forceinline__ void codes_from_dem(SM& sm, const float* __restrict__ dem, uint8_t* __restrict__ dirs,
                                               const DemInfo& dm, int64_t y0, int64_t x0) {
  constexpr int ZS = BW + 4, ZN = (BW + 4) * (BH + 4);
  constexpr int HS = BW + 2, HN = (BW + 2) * (BH + 2);
  const int tid = threadIdx.x;
  const int64_t H = dm.H, W = dm.W;
  const float* Z = dem + dm.off;
  const float kNaN = __builtin_nanf("");
  for (int i = tid; i < ZN; i += NT) {
    const int lr = i / ZS, lc = i - lr * ZS;
    const int64_t gy = y0 + lr - 2, gx = x0 + lc - 2;
    sm.z[i] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? Z[gy * W + gx] : kNaN;
  }
  __syncthreads();
  for (int i = tid; i < HN; i += NT) {
    const int lr = i / HS, lc = i - lr * HS;
    const int64_t gy = y0 + lr - 1, gx = x0 + lc - 1;
    uint8_t k = kOutside;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const float* p = &sm.z[(lr + 1) * ZS + lc + 1];
      const float c = p[0];
      if (__builtin_isnan(c)) {
        k = kNoData;
      } else if (gy == 0 || gx == 0 || gy == H - 1 || gx == W - 1) {
        k = kNone;
      } else {
        const float n0 = p[1], n1 = p[1 - ZS], n2 = p[-ZS], n3 = p[-1 - ZS];
        const float n4 = p[-1], n5 = p[ZS - 1], n6 = p[ZS], n7 = p[ZS + 1];
        const bool nanadj = __builtin_isnan(n0) | __builtin_isnan(n1) | __builtin_isnan(n2) |
                            __builtin_isnan(n3) | __builtin_isnan(n4) | __builtin_isnan(n5) |
                            __builtin_isnan(n6) | __builtin_isnan(n7);
        k = nanadj ? kNone : lowest8(c, n0, n1, n2, n3, n4, n5, n6, n7);
      }
    }
    sm.code[i] = k;
  }
  __syncthreads();
  uint8_t* D = dirs + dm.off;
  for (int i = tid; i < BW * BH; i += NT) {
    const int r = i / BW, c = i - r * BW;
    if (y0 + r < H && x0 + c < W) D[(y0 + r) * W + x0 + c] = sm.code[(r + 1) * HS + c + 1];
  }
}

struct BlockGeo {
  DemInfo dm;
  int64_t y0, x0;       // block origin
  int64_t ty0, tx0;     // global tile coordinates of the block's first tile
  int bw, bh;           // block extent clipped to the DEM
};

template <int BW, int BH, int TS>
__device__ __forceinline__ BlockGeo block_geo(const DemTable& tab, int64_t blk) {
  BlockGeo b;
  b.dm = dem_of_block(tab, blk);
  // block index within its DEM: below 2^32 (a DEM has fewer than 2^32 cells)
  const uint32_t lb = (uint32_t)(blk - b.dm.blk0);
  const uint32_t by = lb / (uint32_t)b.dm.BX, bx = lb - by * (uint32_t)b.dm.BX;
  b.y0 = (int64_t)by * BH;
  b.x0 = (int64_t)bx * BW;
  b.ty0 = (int64_t)by * (BH / TS);
  b.tx0 = (int64_t)bx * (BW / TS);
  b.bh = (int)min((int64_t)BH, (int64_t)b.dm.H - b.y0);
  b.bw = (int)min((int64_t)BW, (int64_t)b.dm.W - b.x0);
  return b;
}

// Values: V = uint32_t for counts (w = 1; integer sums, so the result does
// not depend on the order of the atomic additions), V = double for weights
// (fp64 sums: the rounding of any order is far below float32 output
// precision).  The pass writes the tile-local areas to the output and the
// perimeter records of every tile; the finalising pass adds the inflows.
template <int BW, int BH, int TS, typename V, int CPT>
__global__ __launch_bounds__(BW * BH / CPT) __attribute__((amdgpu_waves_per_eu(CPT == 8 ? 8 : 1))) void k_block_emit(
    const uint8_t* __restrict__ dirs, const float* __restrict__ w, DemTable tab, int64_t nblocks, int cap,
    uint8_t* __restrict__ ex_code, uint16_t* __restrict__ rl, void* __restrict__ ex_val, void* __restrict__ out,
    float* __restrict__ out_lo, uint32_t* __restrict__ status, const float* __restrict__ dem,
    uint8_t* __restrict__ dirs_out, int64_t first) {
  constexpr bool kCount = std::is_same<V, uint32_t>::value;
  using EV = std::conditional_t<kCount, uint64_t, double>;  // exit values for the resolve
  constexpr int NC = BW * BH;
  constexpr int NT = NC / CPT;
  constexpr int HS = BW + 2;
  constexpr int TPX = BW / TS, TPY = BH / TS;  // tiles per block row / column
  static_assert(TPX * TS == BW && TPY * TS == BH, "block of whole tiles");
  __shared__ DblSmem<BW, BH, V> sm;
  const BlockGeo g = block_geo<BW, BH, TS>(tab, first + xcd_tile(blockIdx.x, nblocks));
  const int tid = threadIdx.x;
  const int64_t W = g.dm.W;
  const int64_t base = g.dm.off + g.y0 * W + g.x0;  // the block's first cell
  D8_STAMP(0, 0);
  float wv[kCount ? 1 : CPT];
  if (!kCount) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int c = tid + k * NT;
      const int r = c / BW, col = c % BW;
      wv[k] = (w && r < g.bh && col < g.bw) ? w[base + r * W + col] : 1.0f;
    }
  }
  if (dem) {
    codes_from_dem<BW, BH, NT>(sm, dem, dirs_out, g.dm, g.y0, g.x0);
  } else {
    load_halo<BW, BH, NT>(sm.code, dirs, g.dm, g.y0, g.x0, g.bw);
    __syncthreads();
  }
  D8_STAMP(0, 1);

  // Setup: in-tile target (ancestor at distance 1), the target's own target
  // (distance 2) and the initial value.  Every code a thread needs is read
  // before any is used (one LDS round trip per distance, not one per cell).
  // Only blocks on the DEM's border can have targets off the grid.
  const bool border = g.y0 == 0 || g.x0 == 0 || g.y0 + BH >= g.dm.H || g.x0 + BW >= g.dm.W;
  // Cells are taken in batches of SB (register pressure).
  constexpr int SB = CPT < 4 ? CPT : 4;
  bool bad = false;
  static_assert(BW * BH <= 16384, "link offsets in 16 bits");
  uint32_t a[CPT];  // 2^j-th ancestor as a link byte offset, or kNoAnc
  uint16_t a1[CPT];
  V v0[CPT];
  bool more = false;
#pragma unroll
  for (int h = 0; h < CPT; h += SB) {
    uint32_t cd[SB], td[SB], ud[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int c = tid + (h + q) * NT;
      const int r = c / BW, col = c % BW;
      cd[q] = sm.code[(r + 1) * HS + col + 1];
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int c = tid + (h + q) * NT;
      const int r = c / BW, col = c % BW;
      const uint32_t d = cd[q] & 7u;
      td[q] = sm.code[(r + 1 + ddr_t(d)) * HS + col + 1 + ddc_t(d)];
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int c = tid + (h + q) * NT;
      const int r = c / BW, col = c % BW;
      const uint32_t d = cd[q] & 7u, e = td[q] & 7u;
      // two steps can leave the halo: clamped (the code read is then unused)
      const int ur = min(max(r + 1 + ddr_t(d) + ddr_t(e), 0), BH + 1);
      const int uc = min(max(col + 1 + ddc_t(d) + ddc_t(e), 0), BW + 1);
      ud[q] = sm.code[ur * HS + uc];
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int k = h + q;
      const int c = tid + k * NT;
      const int r = c / BW, col = c % BW;
      const uint32_t code = cd[q], tcode = td[q];
      // (bitwise & and | on the flags: no branches)
      const bool ok = (r < g.bh) & (col < g.bw) & (code != kNoData);
      const uint32_t d = code & 7u;
      const int dr = ddr_t(d), dc = ddc_t(d);
      const int ta = r / TS, tb = col / TS;
      const int th = min(TS, g.bh - ta * TS), tw = min(TS, g.bw - tb * TS);
      const int tr = r - ta * TS + dr, tc = col - tb * TS + dc;
      const bool drains = ok & (code < 8u);
      const bool inside = drains & ((unsigned)tr < (unsigned)th) & ((unsigned)tc < (unsigned)tw);
      bad |= ok & ((code > 8u) | (drains & (tcode == kNoData)));
      if (border) {
        // local row / column of the target against the DEM's edges
        const int gr = r + dr, gc = col + dc;
        bad |= drains & !inside &
               (((g.y0 == 0) & (gr < 0)) | ((g.y0 + BH >= g.dm.H) & (gr >= g.bh)) | ((g.x0 == 0) & (gc < 0)) |
                ((g.x0 + BW >= g.dm.W) & (gc >= g.bw)));
      }
      const bool has1 = inside & (tcode != kNoData);
      // the target's own in-tile target, by the same rule
      const uint32_t e = tcode & 7u;
      const int ur = tr + ddr_t(e), uc = tc + ddc_t(e);
      const bool has2 = has1 & (tcode < 8u) & ((unsigned)ur < (unsigned)th) & ((unsigned)uc < (unsigned)tw) &
                        (ud[q] != kNoData);
      a1[k] = has1 ? (uint16_t)(c + dr * BW + dc) : kNoAnc;
      a[k] = has2 ? 4u * (uint32_t)(c + (dr + ddr_t(e)) * BW + dc + ddc_t(e)) : (uint32_t)kNoAnc;
      more |= has2;
      if constexpr (kCount)
        v0[k] = ok ? 1u : 0u;
      else
        v0[k] = ok ? (double)wv[k] : 0.0;
      sm.val[c] = v0[k];
      const uint32_t root = has2 ? a[k] : 4u * (uint32_t)(has1 ? a1[k] : (uint16_t)c);
      sm.link[c] = a[k] | (root << 16);
    }
  }
  if (bad) set_status(status, kStBadDir);  // invalid code, or a target off the grid / into NoData
  __shared__ RoundFlag rf;
  if (threadIdx.x == 0) rf.f[0] = rf.f[1] = 0;
  __syncthreads();
  D8_STAMP(0, 2);

  // Round 0 of the doubling: every cell adds its initial value to its target
  // (the links already name the distance-2 ancestors).
#pragma unroll
  for (int k = 0; k < CPT; ++k)
    if (a1[k] != kNoAnc) atomicAdd(&sm.val[a1[k]], v0[k]);
  if (more) rf.f[0] = 1;
  __syncthreads();

  // Rounds 1, 2, ...  Reads of a round (own value, ancestor's link word) all
  // happen before the barrier, updates after it.  The saturating pointer
  // becomes the ancestor's saturating pointer when the exact one runs out.
  const int max_rounds = 2 + 31 - __builtin_clz((unsigned)(TS * TS));
  for (int round = 1; rf.f[(round - 1) & 1]; ++round) {
    if (round > max_rounds) {
      set_status(status, kStCycle);  // a cycle never runs out of ancestors
      break;
    }
    V v[CPT];
    uint32_t nl[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (a[k] != kNoAnc) {
        v[k] = sm.val[tid + k * NT];
        nl[k] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(sm.link) + a[k]);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) rf.f[(round + 1) & 1] = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      // two adjacent lanes adding to the same ancestor add once (pairs
      // alternate with k; lane 0 of a wave has no left neighbour)
      const bool valid = a[k] != kNoAnc;
      const bool right = (((tid + k) & 1) != 0) & ((tid & 63) != 0);
      const bool dup = merge_pair_add<V>(a[k], valid, right, v[k]);
      if (valid) {
        if (!dup) atomicAdd(reinterpret_cast<V*>(reinterpret_cast<char*>(sm.val) + a[k] * (sizeof(V) / 4)), v[k]);
        // the new exact ancestor; once it runs out, the ancestor's word as a
        // whole (its exact half is kNoAnc too, its high half the root)
        const uint32_t na = nl[k] & 0xFFFFu;
        a[k] = na;
        sm.link[tid + k * NT] = na == kNoAnc ? nl[k] : na * 0x10001u;
      }
    }
    // any ancestor left: the AND of the pointers is kNoAnc only if all are
    uint32_t all = kNoAnc;
#pragma unroll
    for (int k = 0; k < CPT; ++k) all &= a[k];
    if (all != kNoAnc) rf.f[round & 1] = 1;
    __syncthreads();
  }
  __syncthreads();
  D8_STAMP(0, 3);

  // Tile-local areas.
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    const int r = c / BW, col = c % BW;
    if (r < g.bh && col < g.bw) {
      const int64_t o = base + r * W + col;
      if constexpr (kCount) {
        static_cast<uint32_t*>(out)[o] = sm.val[c];
      } else {
        const double x = sm.val[c];
        const float hi = (float)x;
        static_cast<float*>(out)[o] = hi;
        if (out_lo) out_lo[o] = (float)(x - (double)hi);
      }
    }
  }
  D8_STAMP(0, 4);
  // Perimeter records of every tile of the block (Alg. 4): exit values, and
  // for each receiver the exit its in-tile path leaves by.
  for (int idx = tid; idx < TPX * TPY * cap; idx += NT) {
    const int tl = idx / cap, j = idx - tl * cap;
    const int ta = tl / TPX, tb = tl - ta * TPX;
    const int th = g.bh - ta * TS, tw = g.bw - tb * TS;
    if (th <= 0 || tw <= 0) continue;  // tile beyond the DEM edge
    const int thc = min(TS, th), twc = min(TS, tw);
    const int64_t sb = (g.dm.tile0 + (g.ty0 + ta) * g.dm.TX + g.tx0 + tb) * cap;
    uint8_t ec = 0xFF;
    if (j < perim_count(twc, thc)) {
      int lr, lc;
      perim_cell(j, twc, thc, lr, lc);
      const int r = ta * TS + lr, col = tb * TS + lc;
      const uint32_t code = sm.code[(r + 1) * HS + col + 1];
      if (code < 8u) {
        const int tr = lr + ddr_t(code), tc = lc + ddc_t(code);
        if (!(tr >= 0 && tr < thc && tc >= 0 && tc < twc)) {
          const int64_t gy = g.y0 + r + ddr_t(code), gx = g.x0 + col + ddc_t(code);
          if (gy >= 0 && gy < g.dm.H && gx >= 0 && gx < g.dm.W &&
              sm.code[(r + 1 + ddr_t(code)) * HS + col + 1 + ddc_t(code)] != kNoData) {
            ec = (uint8_t)code;
            static_cast<EV*>(ex_val)[sb + j] = (EV)sm.val[r * BW + col];
          }
        }
      }
      if (code != kNoData && (input_mask<BW>(sm.code, r, col) & outside_dirs(lr, lc, twc, thc))) {
        // Receiver: the root of its in-tile path is the exit it leaves by,
        // unless the path ends at an outlet.
        const int root = (int)(sm.link[r * BW + col] >> 18);  // byte offset / 4
        const int R = root / BW, C = root % BW;
        const uint32_t k2 = sm.code[(R + 1) * HS + C + 1];
        uint16_t link = 0xFFFF;
        if (k2 < 8u) {
          const int64_t gy = g.y0 + R + ddr_t(k2), gx = g.x0 + C + ddc_t(k2);
          if (gy >= 0 && gy < g.dm.H && gx >= 0 && gx < g.dm.W &&
              sm.code[(R + 1 + ddr_t(k2)) * HS + C + 1 + ddc_t(k2)] != kNoData)
            link = (uint16_t)perim_slot(R - ta * TS, C - tb * TS, twc, thc);
        }
        rl[sb + j] = link;
      }
    }
    ex_code[sb + j] = ec;
  }
  D8_STAMP(0, 5);
}

// Offsets of the eight directions in a row-major array of row stride HS, as
// signed bytes packed into one word.
__host__ __device__ constexpr uint64_t hoff_table(int hs) {
  const int o[8] = {1, 1 - hs, -hs, -hs - 1, -1, hs - 1, hs, hs + 1};
  uint64_t t = 0;
  for (int i = 0; i < 8; ++i) t |= (uint64_t)(uint8_t)(int8_t)o[i] << (8 * i);
  return t;
}
template <int HS>
__device__ __forceinline__ int hoff(uint32_t d) {
  if constexpr (HS + 1 <= 127) {
    constexpr uint64_t t = hoff_table(HS);
    return (int)(int8_t)(uint8_t)(t >> (8 * d));
  } else {
    return ddr_t(d) * HS + ddc_t(d);
  }
}

// ------------------------------------------------------- finalising pass --
// Alg. 7-8: each receiver's incoming area (the resolved areas of the exits of
// other tiles that drain into it, summed per receiver slot by the down pass of
// the super-block resolve) is added to every cell on its downstream path
// inside the tile.  The emit pass already wrote the tile-local areas, so
// only the cells downstream of receivers change: each receiver with inflow
// walks its path accumulating into an LDS array (paths may share cells; the
// sums are exact for counts and fp64 for weights), then the touched cells of
// the output are updated.
// Before the walks, every perimeter cell whose step leaves the tile gets the
// outlet code in the tile's LDS copy of the codes, so that a walk stops there
// after adding and never needs its coordinates: it moves by the in-tile offset
// of the code alone.
template <int TS, int NRX>
__device__ __forceinline__ void mark_tile_exits(uint8_t* code, const int (&hr)[NRX], int th, int tw) {
#pragma unroll
  for (int q = 0; q < NRX; ++q) {
    if (hr[q] < 0) continue;
    const uint32_t k = code[hr[q]];
    if (k < 8u) {
      const int nr = hr[q] / TS + ddr_t(k), nc = hr[q] % TS + ddc_t(k);
      if ((unsigned)nr >= (unsigned)th || (unsigned)nc >= (unsigned)tw) code[hr[q]] = kNone;
    }
  }
}

// Walks of the finalising pass: each receiver q with inflow xr[q] adds it at
// every cell of its in-tile path (row stride TS), atomically into Y.  The
// walk loop runs while any lane of the wave is still walking (a uniform
// test), and a lane's stop conditions are folded into one flag rather than
// taken as separate branches, so that the loop does little exec-mask work.
template <int TS, typename V, int NRX>
__device__ __forceinline__ void fixup_walks(const uint8_t* code, V* Y, const int (&hr)[NRX], const V (&xr)[NRX]) {
  constexpr int NC = TS * TS;
#pragma unroll
  for (int q = 0; q < NRX; ++q) {
    const V x = xr[q];
    bool live = hr[q] >= 0 && x != (V)0;
    int p = live ? hr[q] : 0;
    // bounded: a cycle never ends
    V xc = x;  // what this lane carries (its own inflow and any it absorbed)
    const uint32_t lane = threadIdx.x & 63u;
    // right lanes of the pairs on even and on odd steps (lane 0 of the wave
    // has no left neighbour)
    const bool right_even = (lane & 1u) != 0u;
    const bool right_odd = ((lane & 1u) == 0u) & (lane != 0u);
    for (int n = 0; n < NC && __builtin_amdgcn_ballot_w64(live); ++n) {
      const uint32_t k = code[p];
      {
        // Two lanes at the same cell at the same step follow the same path
        // from here on: the right one of an adjacent lane pair hands its
        // value to the left one and stops.  Pairs alternate by step
        // ((0,1), (2,3), ... then (1,2), (3,4), ...), so a lane is never
        // both absorbing and absorbed in one step.  The shifts write 0 where
        // the source lane is beyond the wave (bound_ctrl): lane 0 is never a
        // right lane, and lane 63 gains 0.
        const int pk = live ? p : -1;
        const int pl = __builtin_amdgcn_mov_dpp(pk, 0x138, 0xF, 0xF, true);  // lane - 1 (wave_shr:1)
        const bool right = (n & 1) ? right_odd : right_even;
        const bool dup = right & live & (pl == p);
        const V give = dup ? xc : (V)0;
        if constexpr (std::is_same<V, uint32_t>::value) {
          xc += (uint32_t)__builtin_amdgcn_mov_dpp((int)give, 0x130, 0xF, 0xF, true);  // from lane + 1 (wave_shl:1)
        } else {
          const uint64_t gb = __builtin_bit_cast(uint64_t, give);
          const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)gb, 0x130, 0xF, 0xF, true);
          const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(gb >> 32), 0x130, 0xF, 0xF, true);
          xc += __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
        }
        live = live & !dup;
      }
      const bool add = live & (k < kOutside);  // not a NoData target (flagged by the emit pass)
      if (add) atomicAdd(&Y[p], xc);
      // on to the next cell unless this one is an outlet, an exit of the tile
      // (marked as an outlet) or carries an invalid code (flagged by the emit
      // pass)
      live = add & (k < 8u);
      p = live ? p + hoff<TS>(k) : p;
    }
  }
}

template <int TS, typename V>
__global__ __launch_bounds__(256) void k_fixup(const uint8_t* __restrict__ dirs, DemTable tab, int64_t ntiles,
                                               int cap, const void* __restrict__ F, void* __restrict__ out,
                                               float* __restrict__ out_lo, int64_t first) {
  constexpr bool kCount = std::is_same<V, uint32_t>::value;
  using FV = std::conditional_t<kCount, uint64_t, double>;  // resolved exit values
  constexpr int NC = TS * TS, NT = 256;
  constexpr int NRX = (4 * TS - 4 + NT - 1) / NT;  // perimeter cells per thread
  // The tile's own codes and inflow sums only (row stride TS): a walk stops
  // by its coordinates where its path leaves the tile, so no halo is kept,
  // and for 64 x 64 counts the block fits eight to a CU's LDS.
  __shared__ __attribute__((aligned(16))) uint8_t code[NC];
  __shared__ __attribute__((aligned(16))) V Y[NC];
  const int tid = threadIdx.x;
  const TileGeo g = tile_geo(tab, first + xcd_tile(blockIdx.x, ntiles), TS);
  D8_STAMP(1, 0);
  // Inflow of every receiver slot, resolved by the super-block pass.
  const FV* X = static_cast<const FV*>(F) + g.tile * cap;
  const int np = perim_count(g.tw, g.th);
  V xr[NRX];
  int hr[NRX];
#pragma unroll
  for (int q = 0; q < NRX; ++q) {
    const int j = tid + q * NT;
    xr[q] = 0;
    hr[q] = -1;
    if (j < np) {
      int lr, lc;
      perim_cell(j, g.tw, g.th, lr, lc);
      xr[q] = (V)X[j];
      hr[q] = lr * TS + lc;
    }
  }
  constexpr int KPT = NC / NT;
  static_assert(KPT * NT == NC, "whole tile per pass");
  const int64_t base = g.dm.off + g.y0 * g.dm.W + g.x0;
  const int64_t W = g.dm.W;
  // A whole 64 x 64 tile whose rows are 4-cell aligned: each thread moves
  // groups of 4 cells (one 32-bit word of codes, one 16-byte vector of output
  // values, and of low parts for weights) instead of single cells.
  if constexpr (TS == 64) {
    constexpr int GPR = TS / 4, KG = NC / 4 / NT;  // groups per row, per thread
    const uintptr_t al = reinterpret_cast<uintptr_t>(out) | (kCount ? 0 : reinterpret_cast<uintptr_t>(out_lo));
    if (g.tw == TS && g.th == TS && ((base | W) & 3) == 0 && (al & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(dirs) & 3) == 0) {
      using OV4 = std::conditional_t<kCount, uint4, float4>;
      using OS = std::conditional_t<kCount, uint32_t, float>;
      const uint32_t* D = reinterpret_cast<const uint32_t*>(dirs + base);
      OS* O = static_cast<OS*>(out) + base;
      float* L = (!kCount && out_lo) ? out_lo + base : nullptr;
      uint32_t cw[KG];
      OV4 o4[KG];
      float4 l4[kCount ? 1 : KG];
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const int j = tid + q * NT, r = j / GPR, c4 = (j % GPR) * 4;
        cw[q] = D[(r * W + c4) / 4];
        // counts: the tile-local values are read after the walks, only for
        // groups a walk touched
        if constexpr (!kCount) {
          o4[q] = *reinterpret_cast<const OV4*>(O + r * W + c4);
          l4[q] = L ? *reinterpret_cast<const float4*>(L + r * W + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const int j = tid + q * NT;
        reinterpret_cast<uint32_t*>(code)[j] = cw[q];
        if constexpr (kCount) {
          reinterpret_cast<uint4*>(Y)[j] = make_uint4(0u, 0u, 0u, 0u);
        } else {
          reinterpret_cast<double2*>(Y)[2 * j] = make_double2(0.0, 0.0);
          reinterpret_cast<double2*>(Y)[2 * j + 1] = make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
      mark_tile_exits<TS, NRX>(code, hr, g.th, g.tw);
      __syncthreads();
      D8_STAMP(1, 1);
      fixup_walks<TS, V, NRX>(code, Y, hr, xr);
      __syncthreads();
      D8_STAMP(1, 2);
      if constexpr (kCount) {
        // touched groups: read the 4 tile-local values (loads issued for all
        // groups first), add, write the group back whole
        uint4 y[KG];
        bool tq[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          const int j = tid + q * NT, r = j / GPR, c4 = (j % GPR) * 4;
          y[q] = reinterpret_cast<const uint4*>(Y)[j];
          tq[q] = (y[q].x | y[q].y | y[q].z | y[q].w) != 0u;
          if (tq[q]) o4[q] = *reinterpret_cast<const OV4*>(O + r * W + c4);
        }
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          const int j = tid + q * NT, r = j / GPR, c4 = (j % GPR) * 4;
          if (tq[q])
            *reinterpret_cast<OV4*>(O + r * W + c4) =
                make_uint4(o4[q].x + y[q].x, o4[q].y + y[q].y, o4[q].z + y[q].z, o4[q].w + y[q].w);
        }
      }
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const int j = tid + q * NT, r = j / GPR, c4 = (j % GPR) * 4;
        const int64_t e = r * W + c4;
        if constexpr (kCount) {
          (void)e;
        } else {
          const double2 ya = reinterpret_cast<const double2*>(Y)[2 * j];
          const double2 yb = reinterpret_cast<const double2*>(Y)[2 * j + 1];
          const double y[4] = {ya.x, ya.y, yb.x, yb.y};
          const float ov[4] = {o4[q].x, o4[q].y, o4[q].z, o4[q].w};
          const float lv[4] = {l4[q].x, l4[q].y, l4[q].z, l4[q].w};
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (y[t] != 0.0) {
              const double x = (double)ov[t] + (double)lv[t] + y[t];
              const float hi = (float)x;
              O[e + t] = hi;
              if (L) L[e + t] = (float)(x - (double)hi);
            }
          }
        }
      }
      D8_STAMP(1, 3);
      D8_STAMP(1, 4);
      D8_STAMP(1, 5);
      return;
    }
  }
  using OV = std::conditional_t<kCount, uint32_t, float>;
  OV o[KPT];
  float l[KPT];
  uint8_t cd[KPT];
  {
    const OV* O = static_cast<const OV*>(out) + base;
    const uint8_t* D = dirs + base;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int i = tid + k * NT;
      const bool in = i / TS < g.th && i % TS < g.tw;
      o[k] = in ? O[(i / TS) * W + i % TS] : (OV)0;
      l[k] = (!kCount && out_lo && in) ? out_lo[base + (i / TS) * W + i % TS] : 0.0f;
      cd[k] = in ? D[(i / TS) * W + i % TS] : kOutside;
    }
  }
#pragma unroll
  for (int k = 0; k < KPT; ++k) {
    code[tid + k * NT] = cd[k];
    Y[tid + k * NT] = 0;
  }
  __syncthreads();
  mark_tile_exits<TS, NRX>(code, hr, g.th, g.tw);
  __syncthreads();
  D8_STAMP(1, 1);
  // Walks: add the inflow at every cell of the receiver's in-tile path.
  fixup_walks<TS, V, NRX>(code, Y, hr, xr);
  __syncthreads();
  D8_STAMP(1, 2);
  // The tile-local values written by the emit pass were fetched at the start
  // (their latency overlaps the walks); only the touched cells are stored.
  V y[KPT];
#pragma unroll
  for (int k = 0; k < KPT; ++k) y[k] = Y[tid + k * NT];
  D8_STAMP(1, 3);
  if constexpr (kCount) {
    uint32_t* O = static_cast<uint32_t*>(out) + base;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int i = tid + k * NT;
      if (y[k]) O[(i / TS) * W + i % TS] = o[k] + y[k];
    }
  } else {
    float* O = static_cast<float*>(out) + base;
    float* L = out_lo ? out_lo + base : nullptr;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int i = tid + k * NT;
      if (y[k] != 0.0) {
        const int64_t q = (i / TS) * W + i % TS;
        const double x = (double)o[k] + (double)l[k] + y[k];
        const float hi = (float)x;
        O[q] = hi;
        if (L) L[q] = (float)(x - (double)hi);
      }
    }
  }
  D8_STAMP(1, 4);
  D8_STAMP(1, 5);
}

// --------------------------------------------- backward: in-tile path sums --
// The adjoint of Eq. (1): G(c) = g(c) + G(target(c)).  Inside a tile this is
// the sum of g along c's path to the tile root, computed by pointer jumping
// (pull form, no atomics): in round j a cell adds the partial sum of its
// 2^j-th ancestor and jumps to that ancestor's ancestor.  fp64 partial sums in
// a fixed order, so the result is deterministic.  Block and link layout as in
// k_block_emit (the saturating root field ends at the tile root).
//   emit pass   writes, for every receiver, its path sum (rg) and the exit it
//               leaves by (rl), and marks exits in ex_code; for every cell,
//               its in-tile path sum as a float32 pair (high part into the
//               output, low part into blo: the pair keeps the fp64 sum to
//               2^-48 of its magnitude) and the perimeter index of the exit
//               its path leaves by (broot);
//   final pass  adds H(root exit), the resolved path sum beyond the tile, to
//               every cell whose path leaves the tile (a streaming pass: the
//               in-tile sums are not recomputed).
template <int BW, int BH>
struct BwdSmem {
  double S[BW * BH];
  uint32_t link[BW * BH];
  uint8_t code[(BW + 2) * (BH + 2)];
};

template <int BW, int BH, int TS, int CPT>
__global__ __launch_bounds__(BW * BH / CPT) __attribute__((amdgpu_waves_per_eu(CPT == 8 ? 6 : 1))) void k_block_bwd(
    const uint8_t* __restrict__ dirs, const float* __restrict__ gin, DemTable tab, int64_t nblocks, int cap,
    uint8_t* __restrict__ ex_code, uint16_t* __restrict__ rl, double* __restrict__ rg,
    float* __restrict__ blo, uint16_t* __restrict__ broot, float* __restrict__ out, uint32_t* __restrict__ status) {
  constexpr int NC = BW * BH;
  constexpr int NT = NC / CPT;
  constexpr int HS = BW + 2;
  constexpr int TPX = BW / TS, TPY = BH / TS;
  static_assert(TPX * TS == BW && TPY * TS == BH, "block of whole tiles");
  __shared__ BwdSmem<BW, BH> sm;
  const BlockGeo g = block_geo<BW, BH, TS>(tab, xcd_tile(blockIdx.x, nblocks));
  const int tid = threadIdx.x;
  const int64_t W = g.dm.W;
  const int64_t base = g.dm.off + g.y0 * W + g.x0;
  double s[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    const int r = c / BW, col = c % BW;
    s[k] = (r < g.bh && col < g.bw) ? (double)gin[base + r * W + col] : 0.0;
  }
  load_halo<BW, BH, NT>(sm.code, dirs, g.dm, g.y0, g.x0, g.bw);
  __syncthreads();

  const bool border = g.y0 == 0 || g.x0 == 0 || g.y0 + BH >= g.dm.H || g.x0 + BW >= g.dm.W;
  uint16_t a[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    const int r = c / BW, col = c % BW;
    const uint32_t code = sm.code[(r + 1) * HS + col + 1];
    const bool ok = r < g.bh && col < g.bw && code != kNoData;
    const uint32_t d = code & 7u;
    const int dr = ddr_t(d), dc = ddc_t(d);
    const int ta = r / TS, tb = col / TS;
    const int th = min(TS, g.bh - ta * TS), tw = min(TS, g.bw - tb * TS);
    const int tr = r - ta * TS + dr, tc = col - tb * TS + dc;
    const bool drains = ok && code < 8u;
    const bool inside = drains && tr >= 0 && tr < th && tc >= 0 && tc < tw;
    const uint8_t tcode = sm.code[(r + 1 + dr) * HS + col + 1 + dc];
    bool bad = ok && (code > 8u || (drains && tcode == kNoData));
    if (border)
      bad |= drains && !inside &&
             (g.y0 + r + dr < 0 || g.y0 + r + dr >= g.dm.H || g.x0 + col + dc < 0 || g.x0 + col + dc >= g.dm.W);
    if (bad) set_status(status, kStBadDir);
    a[k] = (inside && tcode != kNoData) ? (uint16_t)(c + dr * BW + dc) : kNoAnc;
    if (!ok) s[k] = 0.0;
    sm.S[c] = s[k];
    sm.link[c] = (uint32_t)a[k] | ((uint32_t)(a[k] != kNoAnc ? a[k] : (uint16_t)c) << 16);
  }
  __syncthreads();

  const int max_rounds = 2 + 31 - __builtin_clz((unsigned)(TS * TS));
  __shared__ RoundFlag rf;
  if (threadIdx.x == 0) rf.f[0] = rf.f[1] = 0;
  __syncthreads();
  for (int round = 0;; ++round) {
    double sa[CPT];
    uint32_t nl[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (a[k] != kNoAnc) {
        sa[k] = sm.S[a[k]];
        nl[k] = sm.link[a[k]];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) rf.f[(round + 1) & 1] = 0;
    bool more = false;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (a[k] != kNoAnc) {
        const int c = tid + k * NT;
        s[k] += sa[k];
        sm.S[c] = s[k];
        const uint16_t na = (uint16_t)(nl[k] & 0xFFFFu);
        const uint32_t root = na != kNoAnc ? (uint32_t)na : (nl[k] >> 16);
        a[k] = na;
        sm.link[c] = (uint32_t)na | (root << 16);
        more |= na != kNoAnc;
      }
    }
    if (more) rf.f[round & 1] = 1;
    __syncthreads();
    if (!rf.f[round & 1]) break;
    if (round >= max_rounds) {
      set_status(status, kStCycle);
      break;
    }
  }
  __syncthreads();

  // Slot of the exit at block cell `root` if that cell is an exit of its
  // tile, else -1.
  auto exit_slot = [&](int root, int64_t& sl) -> bool {
    const int R = root / BW, C = root % BW;
    const int ta = R / TS, tb = C / TS;
    const int thc = min(TS, g.bh - ta * TS), twc = min(TS, g.bw - tb * TS);
    const uint32_t k2 = sm.code[(R + 1) * HS + C + 1];
    if (k2 >= 8u) return false;
    const int tr = R - ta * TS + ddr_t(k2), tc = C - tb * TS + ddc_t(k2);
    if (tr >= 0 && tr < thc && tc >= 0 && tc < twc) return false;  // not an exit
    const int64_t gy = g.y0 + R + ddr_t(k2), gx = g.x0 + C + ddc_t(k2);
    if (gy < 0 || gy >= g.dm.H || gx < 0 || gx >= g.dm.W ||
        sm.code[(R + 1 + ddr_t(k2)) * HS + C + 1 + ddc_t(k2)] == kNoData)
      return false;
    sl = (g.dm.tile0 + (g.ty0 + ta) * g.dm.TX + g.tx0 + tb) * cap +
         perim_slot(R - ta * TS, C - tb * TS, twc, thc);
    return true;
  };

  // Per cell: the in-tile path sum and the exit its path leaves by.
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    const int r = c / BW, col = c % BW;
    if (r < g.bh && col < g.bw) {
      const int64_t o = base + r * W + col;
      uint16_t e = 0xFFFF;
      int64_t sl;
      if (sm.code[(r + 1) * HS + col + 1] != kNoData && exit_slot((int)(sm.link[c] >> 16), sl))
        e = (uint16_t)(sl - (g.dm.tile0 + (g.ty0 + r / TS) * g.dm.TX + g.tx0 + col / TS) * cap);
      const float hi = (float)s[k];
      out[o] = hi;
      blo[o] = (float)(s[k] - (double)hi);
      broot[o] = e;
    }
  }
  {
    for (int idx = tid; idx < TPX * TPY * cap; idx += NT) {
      const int tl = idx / cap, j = idx - tl * cap;
      const int ta = tl / TPX, tb = tl - ta * TPX;
      const int th = g.bh - ta * TS, tw = g.bw - tb * TS;
      if (th <= 0 || tw <= 0) continue;
      const int thc = min(TS, th), twc = min(TS, tw);
      const int64_t sb = (g.dm.tile0 + (g.ty0 + ta) * g.dm.TX + g.tx0 + tb) * cap;
      uint8_t ec = 0xFF;
      if (j < perim_count(twc, thc)) {
        int lr, lc;
        perim_cell(j, twc, thc, lr, lc);
        const int r = ta * TS + lr, col = tb * TS + lc;
        const int c = r * BW + col;
        const uint32_t code = sm.code[(r + 1) * HS + col + 1];
        int64_t sl;
        if (code < 8u && exit_slot(c, sl)) ec = (uint8_t)code;
        if (code != kNoData && (input_mask<BW>(sm.code, r, col) & outside_dirs(lr, lc, twc, thc))) {
          uint16_t link = 0xFFFF;
          const int root = (int)(sm.link[c] >> 16);
          if (exit_slot(root, sl)) link = (uint16_t)(sl - sb);
          rl[sb + j] = link;
          rg[sb + j] = sm.S[c];
        }
      }
      ex_code[sb + j] = ec;
    }
  }
}

// Final pass of the backward: G(c) = (in-tile path sum: the float32 pair in
// the output and blo) + H(exit c's path leaves by), for the cells whose path
// leaves the tile; fp64 additions, rounded to float32.  The other cells
// already hold their result.
template <int BW, int BH, int TS>
__global__ __launch_bounds__(256) void k_bwd_final(DemTable tab, int64_t nblocks, int cap,
                                                   const float* __restrict__ blo, const uint16_t* __restrict__ broot,
                                                   const double* __restrict__ H0, const double* __restrict__ H1,
                                                   const uint32_t* __restrict__ hdr, float* __restrict__ out) {
  constexpr int NT = 256, CPT = BW * BH / NT;
  const BlockGeo g = block_geo<BW, BH, TS>(tab, xcd_tile(blockIdx.x, nblocks));
  const double* Hb = hdr[2] == 0 ? H0 : H1;
  const int64_t W = g.dm.W;
  const int64_t base = g.dm.off + g.y0 * W + g.x0;
  // all loads of a thread first, then the dependent ones
  uint16_t e[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = threadIdx.x + k * NT;
    const int r = c / BW, col = c % BW;
    e[k] = (r < g.bh && col < g.bw) ? broot[base + r * W + col] : (uint16_t)0xFFFF;
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    if (e[k] == 0xFFFF) continue;
    const int c = threadIdx.x + k * NT;
    const int r = c / BW, col = c % BW;
    const int64_t o = base + r * W + col;
    const int64_t sl = (g.dm.tile0 + (g.ty0 + r / TS) * g.dm.TX + g.tx0 + col / TS) * cap + e[k];
    out[o] = (float)((double)out[o] + (double)blo[o] + Hb[sl]);
  }
}

// ------------------------------------------------------------------ resolve --
// The exit forest: node = exit slot e; parent(e) = the exit reached from e's
// target receiver inside the receiver's tile (none if that path ends at an
// outlet).
__device__ __forceinline__ bool exit_parent(const DemTable& tab, int64_t s, int ts, int cap, uint8_t ec,
                                            const uint16_t* __restrict__ rl, int64_t& tslot, int32_t& parent) {
  const int64_t tile = s / cap;
  const int j = (int)(s - tile * cap);
  const TileGeo g = tile_geo(tab, tile, ts);
  int r, c;
  perim_cell(j, g.tw, g.th, r, c);
  const int64_t gy = g.y0 + r + ddr(ec), gx = g.x0 + c + ddc(ec);
  tslot = slot_of_cell(g.dm, gy, gx, ts, cap);
  const uint16_t link = rl[tslot];
  const int64_t ttile = tslot / cap;
  parent = link == 0xFFFF ? -1 : (int32_t)(ttile * cap + link);
  return parent >= 0;
}

__device__ __forceinline__ void vadd(uint64_t* p, uint64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
__device__ __forceinline__ void vadd(double* p, double v) { unsafeAtomicAdd(p, v); }

// Level-2 node state of the counts resolve: one 64-bit word per node, bits
// 0..39 the sum received, bits 40..62 the children still to arrive (see the
// global resolve below).
constexpr int kL2Shift = 40;
constexpr uint64_t kL2One = 1ull << kL2Shift;
constexpr uint64_t kL2Mask = kL2One - 1;
constexpr uint32_t kL2HasKids = 0x80000000u;
constexpr int kL2Steps = 32;

// ------------------------------------------------ super-block group pass --
// The tile exits of a kSuper x kSuper super-block form a forest whose edges
// stay inside the super-block except at its own exits.  One workgroup
// resolves that forest in LDS (the same doubling as the tile pass, now over
// exit nodes), so the global resolve only sees super-block exits.  The
// downward pass redoes it with the resolved inflows of the super-block's
// receivers added and writes the full area of every tile exit.
template <typename LV>
struct GroupSmem;

template <int TS, typename LV>
struct GroupDims {
  static constexpr int G = kSuper / TS;
  static constexpr int CAP = 4 * TS - 4;
  static constexpr int NN = G * G * CAP;
  // threads: few nodes per thread keep the per-node registers (and with them
  // the waves a CU can hold) in check: 1024 x 4 nodes for 64 x 64 tiles
  static constexpr int NT = TS <= 64 ? 1024 : 512;
  static constexpr int NPT = (NN + NT - 1) / NT;
};

__device__ __forceinline__ void ladd(uint32_t* p, uint32_t v) { atomicAdd(p, v); }
__device__ __forceinline__ void ladd(double* p, double v) { atomicAdd(p, v); }

// Up pass outputs: the super-block exits get dense node ids (in append
// order; count in hdr[3]); l2val[id] = the exit's area within its super-block,
// l2par[id] = the tile exit its target receiver leads to (-1: none), and for
// every tile exit sbroot[slot] = the node id of the super-block exit its path
// reaches (-1: it ends inside the super-block).  The down pass reads the
// resolved node values from F (indexed through sbroot).
template <int TS, typename LV, typename V, bool DOWN>
__global__ __launch_bounds__(TS <= 64 ? 1024 : 512) void k_group(DemTable tab, int64_t nsb, const uint8_t* __restrict__ ex_code,
                                               const uint16_t* __restrict__ rl, V* __restrict__ ex_val,
                                               V* __restrict__ l2val, int32_t* __restrict__ sbroot,
                                               int32_t* __restrict__ l2par, V* __restrict__ l2acc,
                                               uint64_t* __restrict__ l2pend, const V* __restrict__ F,
                                               V* __restrict__ xin, uint32_t* __restrict__ hdr,
                                               uint32_t* __restrict__ status) {
  using D = GroupDims<TS, LV>;
  constexpr int G = D::G, CAP = D::CAP, NN = D::NN, NT = D::NT, NPT = D::NPT;
  __shared__ LV val[NN];
  __shared__ uint32_t link[NN];
  __shared__ uint8_t flag[NN];  // bit 0: an exit of its tile; bit 1: leaves the super-block
  const int tid = threadIdx.x;
  D8_STAMP(DOWN ? 3 : 2, 0);
  const int64_t sbid = xcd_tile(blockIdx.x, nsb);
  const DemInfo dm = dem_of_sb(tab, sbid);
  const uint32_t lsb = (uint32_t)(sbid - dm.sb0);  // below 2^32: a 32-bit division
  const int64_t sby = lsb / (uint32_t)dm.SBX, sbx = lsb - (uint32_t)sby * (uint32_t)dm.SBX;
  const int64_t ty0 = sby * G, tx0 = sbx * G;
  const int64_t y0 = sby * kSuper, x0 = sbx * kSuper;
  const int sbh = (int)min((int64_t)kSuper, (int64_t)dm.H - y0);
  const int sbw = (int)min((int64_t)kSuper, (int64_t)dm.W - x0);

  uint16_t a[NPT];
  int32_t tg[NPT];   // super-block exits: the tile exit the target receiver leads to
  uint16_t tin[NPT];  // exits inside the super-block: the node of their target receiver
  // Loads in three rounds (codes; then exit values and the target receivers'
  // links), each issued for all of a thread's nodes before any is used.
  int64_t sl[NPT];
  uint8_t ec[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tid + k * NT;
    const int tl = n / CAP, j = n - tl * CAP;
    const int ta = tl / G, tb = tl - ta * G;
    const int64_t ty = ty0 + ta, tx = tx0 + tb;
    sl[k] = (dm.tile0 + ty * dm.TX + tx) * CAP + j;
    ec[k] = (n < NN && ty < dm.TY && tx < dm.TX) ? ex_code[sl[k]] : (uint8_t)0xFF;
  }
  int64_t tb_[NPT];   // target receiver's tile slot base
  int rs_[NPT];       // target receiver's perimeter slot
  int tn_[NPT];       // first node of the target tile when it is inside the super-block, else -1
  LV v_[NPT];
  uint16_t lk_[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tid + k * NT;
    v_[k] = 0;
    lk_[k] = 0xFFFF;
    tb_[k] = 0;
    rs_[k] = 0;
    tn_[k] = -1;
    if (ec[k] < 8) {
      const int tl = n / CAP, j = n - tl * CAP;
      const int ta = tl / G, tb = tl - ta * G;
      const int64_t ty = ty0 + ta, tx = tx0 + tb;
      const int th = (int)min((int64_t)TS, (int64_t)dm.H - ty * TS);
      const int tw = (int)min((int64_t)TS, (int64_t)dm.W - tx * TS);
      int r, c;
      perim_cell(j, tw, th, r, c);
      const int64_t gy = ty * TS + r + ddr_t(ec[k]), gx = tx * TS + c + ddc_t(ec[k]);
      // the target receiver's tile and its slot there
      const int64_t tty = gy / TS, ttx = gx / TS;
      const int tth = (int)min((int64_t)TS, (int64_t)dm.H - tty * TS);
      const int ttw = (int)min((int64_t)TS, (int64_t)dm.W - ttx * TS);
      tb_[k] = (dm.tile0 + tty * dm.TX + ttx) * CAP;
      rs_[k] = perim_slot((int)(gy - tty * TS), (int)(gx - ttx * TS), ttw, tth);
      if (gy >= y0 && gy < y0 + sbh && gx >= x0 && gx < x0 + sbw)
        tn_[k] = (int)(((tty - ty0) * G + (ttx - tx0)) * CAP);
      v_[k] = (LV)ex_val[sl[k]];
      lk_[k] = rl[tb_[k] + rs_[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tid + k * NT;
    a[k] = kNoAnc;
    tg[k] = -1;
    tin[k] = kNoAnc;
    if (n >= NN) continue;
    uint8_t f = 0;
    if (ec[k] < 8) {
      f = 1;
      const uint16_t lk = lk_[k];
      if (tn_[k] >= 0) {
        const int tnode = tn_[k];
        if (lk != 0xFFFF) a[k] = (uint16_t)(tnode + lk);
        tin[k] = (uint16_t)(tnode + rs_[k]);
      } else {
        f |= 2;
        // super-block exit: remember the tile exit its target receiver leads
        // to; the global resolve turns it into a parent via that exit's
        // super-block root
        tg[k] = lk == 0xFFFF ? -1 : (int32_t)(tb_[k] + lk);
      }
    }
    val[n] = v_[k];
    link[n] = (uint32_t)a[k] | ((uint32_t)(a[k] != kNoAnc ? a[k] : (uint16_t)n) << 16);
    flag[n] = f;
  }
  __syncthreads();
  D8_STAMP(DOWN ? 3 : 2, 1);
  constexpr int NPB = (4 * kSuper - 4 + NT - 1) / NT;  // super-block perimeter cells per thread
  V xb[NPB];
  int nb[NPB];
  if (DOWN) {
    // Resolved inflow of every receiver on the super-block's border, added at
    // the tile exit its in-tile path leaves by.
    const int P = perim_count(sbw, sbh);
    // Three load rounds, each issued for every cell and direction before any
    // is used: the outside neighbours' exit codes; the super-block roots of
    // those that drain into the border cell; the roots' resolved inflows.
    uint8_t en[NPB][8];
#pragma unroll
    for (int q = 0; q < NPB; ++q) {
      const int i = tid + q * NT;
      int r = 0, c = 0;
      if (i < P) perim_cell(i, sbw, sbh, r, c);
      const int64_t gy = y0 + r, gx = x0 + c;
      const uint32_t out = i < P ? outside_dirs(r, c, sbw, sbh) : 0u;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        en[q][d] = 0xFF;
        const int64_t ny = gy + ddr_t(d), nx = gx + ddc_t(d);
        if ((out & (1u << d)) && ny >= 0 && ny < dm.H && nx >= 0 && nx < dm.W) {
          const uint8_t e = ex_code[slot_of_cell(dm, ny, nx, TS, CAP)];
          // only neighbours whose exit step lands on this border cell count
          en[q][d] = (e < 8 && ddr_t(e) == -ddr_t(d) && ddc_t(e) == -ddc_t(d)) ? e : (uint8_t)0xFF;
        }
      }
    }
    int32_t rt[NPB][8];
#pragma unroll
    for (int q = 0; q < NPB; ++q) {
      const int i = tid + q * NT;
      int r = 0, c = 0;
      if (i < P) perim_cell(i, sbw, sbh, r, c);
      const int64_t gy = y0 + r, gx = x0 + c;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        rt[q][d] = -1;
        if (en[q][d] != 0xFF) rt[q][d] = sbroot[slot_of_cell(dm, gy + ddr_t(d), gx + ddc_t(d), TS, CAP)];
      }
    }
#pragma unroll
    for (int q = 0; q < NPB; ++q) {
      const int i = tid + q * NT;
      xb[q] = 0;
      nb[q] = -1;
      if (i >= P) continue;
      int r, c;
      perim_cell(i, sbw, sbh, r, c);
      const int64_t gy = y0 + r, gx = x0 + c;
      V x = 0;
#pragma unroll
      for (int d = 0; d < 8; ++d)
        if (en[q][d] != 0xFF) x += F[rt[q][d]];
      if (x != (V)0) {
        const int64_t tty = gy / TS, ttx = gx / TS;
        const int tth = (int)min((int64_t)TS, (int64_t)dm.H - tty * TS);
        const int ttw = (int)min((int64_t)TS, (int64_t)dm.W - ttx * TS);
        const int64_t tbase = (dm.tile0 + tty * dm.TX + ttx) * CAP;
        const int rs = perim_slot((int)(gy - tty * TS), (int)(gx - ttx * TS), ttw, tth);
        const uint16_t lk = rl[tbase + rs];
        const int tnode = (int)(((tty - ty0) * G + (ttx - tx0)) * CAP);
        if (lk != 0xFFFF) ladd(&val[tnode + lk], (LV)x);
        xb[q] = x;
        nb[q] = tnode + rs;
      }
    }
    __syncthreads();
  }

  const int max_rounds = 2 + 31 - __builtin_clz((unsigned)NN);
  D8_STAMP(DOWN ? 3 : 2, 2);
  __shared__ RoundFlag rf;
  if (threadIdx.x == 0) rf.f[0] = rf.f[1] = 0;
  __syncthreads();
  for (int round = 0;; ++round) {
    LV v[NPT];
    uint32_t nl[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if (a[k] != kNoAnc) {
        v[k] = val[tid + k * NT];
        nl[k] = link[a[k]];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) rf.f[(round + 1) & 1] = 0;
    bool more = false;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if (a[k] != kNoAnc) {
        ladd(&val[a[k]], v[k]);
        const uint16_t na = (uint16_t)(nl[k] & 0xFFFFu);
        const uint32_t root = na != kNoAnc ? (uint32_t)na : (nl[k] >> 16);
        a[k] = na;
        link[tid + k * NT] = (uint32_t)na | (root << 16);
        more |= na != kNoAnc;
      }
    }
    if (more) rf.f[round & 1] = 1;
    __syncthreads();
    if (!rf.f[round & 1]) break;
    if (round >= max_rounds) {
      set_status(status, kStCycle);
      break;
    }
  }
  __syncthreads();

  D8_STAMP(DOWN ? 3 : 2, 3);
  if (DOWN) {
    // Full areas of the tile exits, then the inflow of every receiver slot of
    // the super-block's tiles (Alg. 7's incoming area): the exits inside the
    // super-block that drain into it plus, on the border, the resolved exits
    // of neighbouring super-blocks.  The finalising pass reads these inflows.
    LV vv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int n = tid + k * NT;
      const bool act = n < NN && (flag[n] & 1);
      vv[k] = act ? val[n] : (LV)0;
      if (act) {
        const int tl = n / CAP, j = n - tl * CAP;
        const int ta = tl / G, tb = tl - ta * G;
        ex_val[(dm.tile0 + (ty0 + ta) * dm.TX + tx0 + tb) * CAP + j] = (V)vv[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (tid + k * NT < NN) val[tid + k * NT] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (tin[k] != kNoAnc && vv[k] != (LV)0) ladd(&val[tin[k]], vv[k]);
#pragma unroll
    for (int q = 0; q < NPB; ++q)
      if (nb[q] >= 0) ladd(&val[nb[q]], (LV)xb[q]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int n = tid + k * NT;
      if (n >= NN) continue;
      const int tl = n / CAP, j = n - tl * CAP;
      const int ta = tl / G, tb = tl - ta * G;
      if (ty0 + ta < dm.TY && tx0 + tb < dm.TX)
        xin[(dm.tile0 + (ty0 + ta) * dm.TX + tx0 + tb) * CAP + j] = (V)val[n];
    }
    D8_STAMP(DOWN ? 3 : 2, 4);
    D8_STAMP(DOWN ? 3 : 2, 5);
    return;
  }
  // Counts: each super-block exit's number of children in the global forest
  // (the walk stage retires them one by one): the exits of neighbouring
  // super-blocks that drain into a border receiver here whose path leads to
  // that exit.  The codes of those neighbours are final (the tile pass wrote
  // them), so they are counted here, in LDS, with no global atomics; the
  // values move to registers and `val` holds the counts meanwhile.
  constexpr bool kKids = std::is_same<V, uint64_t>::value;
  LV vown[kKids ? NPT : 1];
  if constexpr (kKids) {
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int n = tid + k * NT;
      vown[k] = n < NN ? val[n] : (LV)0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (tid + k * NT < NN) val[tid + k * NT] = 0;
    // the border cells' outside neighbours draining into them, and the tile
    // exit each border cell's own path leaves by (loads issued together)
    const int P = perim_count(sbw, sbh);
    uint32_t nkid[NPB];
    int node[NPB];
#pragma unroll
    for (int q = 0; q < NPB; ++q) {
      const int i = tid + q * NT;
      int r = 0, c = 0;
      if (i < P) perim_cell(i, sbw, sbh, r, c);
      const int64_t gy = y0 + r, gx = x0 + c;
      const uint32_t out = i < P ? outside_dirs(r, c, sbw, sbh) : 0u;
      uint8_t e[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        e[d] = 0xFF;
        const int64_t ny = gy + ddr_t(d), nx = gx + ddc_t(d);
        if ((out & (1u << d)) && ny >= 0 && ny < dm.H && nx >= 0 && nx < dm.W)
          e[d] = ex_code[slot_of_cell(dm, ny, nx, TS, CAP)];
      }
      uint16_t lk = 0xFFFF;
      int tnode = 0;
      if (out) {
        const int64_t tty = gy / TS, ttx = gx / TS;
        const int tth = (int)min((int64_t)TS, (int64_t)dm.H - tty * TS);
        const int ttw = (int)min((int64_t)TS, (int64_t)dm.W - ttx * TS);
        const int rs = perim_slot((int)(gy - tty * TS), (int)(gx - ttx * TS), ttw, tth);
        lk = rl[(dm.tile0 + tty * dm.TX + ttx) * CAP + rs];
        tnode = (int)(((tty - ty0) * G + (ttx - tx0)) * CAP);
      }
      uint32_t k = 0;
#pragma unroll
      for (int d = 0; d < 8; ++d)  // a neighbour counts if its exit step lands on this cell
        k += (e[d] < 8 && ddr_t(e[d]) == -ddr_t(d) && ddc_t(e[d]) == -ddc_t(d)) ? 1u : 0u;
      nkid[q] = k;
      node[q] = (k && lk != 0xFFFF) ? tnode + lk : -1;
    }
    __syncthreads();  // every count zeroed
#pragma unroll
    for (int q = 0; q < NPB; ++q) {
      if (node[q] < 0) continue;
      const int rt = (int)(link[node[q]] >> 16);  // the super-block root of that tile exit
      if (flag[rt] & 2) atomicAdd(&val[rt], (LV)nkid[q]);
    }
    __syncthreads();
  }

  // Dense node ids for the super-block exits: one global atomic per
  // workgroup, offsets from an LDS counter.
  uint32_t nsx = 0;  // own nodes that leave the super-block
  uint16_t root[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tid + k * NT;
    const bool act = n < NN && (flag[n] & 1);
    root[k] = act ? (uint16_t)(link[n] >> 16) : (uint16_t)0;
    if (act && (flag[n] & 2)) nsx |= 1u << k;
  }
  __shared__ uint32_t cnt, base;
  if (tid == 0) cnt = 0;
  __syncthreads();
  const uint32_t mine = __builtin_popcount(nsx);
  const uint32_t off = mine ? atomicAdd(&cnt, mine) : 0u;
  __syncthreads();
  if (tid == 0) base = cnt ? atomicAdd(&hdr[3], cnt) : 0u;
  __syncthreads();  // also: every root read before link is reused below
  uint32_t w = base + off;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if (nsx & (1u << k)) {
      const int n = tid + k * NT;
      link[n] = w;  // node id, looked up by the tile exits rooted here
      if constexpr (kKids) {
        l2val[w] = (V)vown[k];
        l2acc[w] = (V)val[n] << kL2Shift;  // children still to arrive, nothing received
      } else {
        l2val[w] = (V)val[n];
        l2acc[w] = 0;
      }
      l2par[w] = tg[k];
      l2pend[w] = 0;
      ++w;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int n = tid + k * NT;
    if (n < NN && (flag[n] & 1)) {
      const int tl = n / CAP, j = n - tl * CAP;
      const int ta = tl / G, tb = tl - ta * G;
      const int r = root[k];
      sbroot[(dm.tile0 + (ty0 + ta) * dm.TX + tx0 + tb) * CAP + j] = (flag[r] & 2) ? (int32_t)link[r] : -1;
    }
  }
  D8_STAMP(DOWN ? 3 : 2, 4);
  D8_STAMP(DOWN ? 3 : 2, 5);
}

// Global resolve over super-block exits.  Node = a super-block exit (dense
// id); its parent is the super-block exit reached from its target receiver
// (via the receiver's tile exit and that exit's super-block root), or none.
// The nodes form a forest and each needs the sum of its subtree (Alg. 6's
// accumulation over the master's graph).  Two stages:
//  1. propagation in dependency order as in Alg. 2, one thread per leaf: a
//     finished node adds its value to its parent and retires one of the
//     parent's pending children with the same atomic; the thread that retires
//     the last one finishes the parent and carries on.  Each edge costs one
//     atomic and no two threads contend for more than a node's children.  A
//     thread stops after kL2Steps nodes (long chains would serialise), parking
//     the node it finished last;
//  2. doubling over what is left (unfinished nodes with the partial sums they
//     have received, and parked nodes with their full values): value V[i]
//     plus a pending increment D[i]; round j folds D_j into V, sends the
//     node's value to its 2^j-th ancestor's D_(j+1) and jumps the ancestor
//     pointer; O(log depth) launches.  Nodes finished in stage 1 take no part.
// Counts keep the stage-1 state in one 64-bit word per node (bits 0..39 the
// sum received, bits 40..62 the children still to arrive); weighted values
// keep an fp64 sum and a pending count whose bit 31 marks a node with
// children, a child's addition being fenced before its retirement.

// Parent ids: -1 root; <= -2 a parked node (parent -(p + 2)).
// Parent of every node (the children were counted by the super-block pass).
__global__ void k_l2_init(const int32_t* __restrict__ sbroot, int32_t* par, const uint32_t* hdr) {
  const int64_t n = hdr[3];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = par[i];  // the tile exit the target receiver leads to
    par[i] = v >= 0 ? sbroot[v] : -1;
  }
}

template <typename V>
__global__ void k_l2_walk(int32_t* par, V* val, V* acc, uint64_t* pend, const uint32_t* __restrict__ hdr) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)hdr[3]) return;
  bool leaf;
  if constexpr (std::is_same<V, uint64_t>::value)
    leaf = acc[i] == 0;  // never received anything: no children
  else
    leaf = *reinterpret_cast<const uint32_t*>(&pend[i]) == 0;
  if (!leaf) return;
  int32_t s = (int32_t)i;
  V v = val[s];
  if constexpr (std::is_same<V, uint64_t>::value) {
    // A node's own value and parent change only by the walk that arrives at
    // it last, so the parent's are read together with the atomic (one round
    // trip per step, not three); they are used only by that last walk.
    int32_t pa = par[s];
    for (int step = 0; pa >= 0; ++step) {
      if (step == kL2Steps) {
        par[s] = -(pa + 2);  // parked: finished, not yet added to its parent
        break;
      }
      const V vp = val[pa];
      const int32_t pp = par[pa];
      const uint64_t old = atomicAdd(&acc[pa], v - kL2One);
      if ((old >> kL2Shift) != 1) break;
      v = vp + (old & kL2Mask) + v;
      val[pa] = v;
      s = pa;
      pa = pp;
    }
  } else {
    for (int step = 0;; ++step) {
      const int32_t pa = par[s];
      if (pa < 0) break;
      if (step == kL2Steps) {
        par[s] = -(pa + 2);  // parked: finished, not yet added to its parent
        break;
      }
      unsafeAtomicAdd(&acc[pa], v);
      __threadfence();
      const uint32_t old = atomicSub(reinterpret_cast<uint32_t*>(&pend[pa]), 1u);
      if ((old & ~kL2HasKids) != 1u) break;
      __threadfence();
      v = val[pa] + __hip_atomic_load(&acc[pa], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      val[pa] = v;
      s = pa;
    }
  }
}

// Appends node i to the list when `take` (one atomic per wave).
__device__ __forceinline__ void append_node(int32_t* list, uint32_t* count, int32_t i, bool take) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(take);
  if (m == 0) return;
  const int lane = (int)__lane_id();
  const int leader = __builtin_ctzll(m);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__builtin_popcountll(m));
  base = __shfl(base, leader);
  if (take) list[base + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1))] = i;
}

// Stage-2 start: ancestor = parent for unfinished and parked nodes (-1 for
// nodes finished and delivered), unfinished nodes fold in what they received,
// pending increments zeroed (they reuse the stage-1 words).  Counts: the
// nodes that take part (parked and unfinished ones: a set closed under
// ancestors, so no other node ever receives an increment) are listed in
// plist (count hdr[4]) and the rounds and the final fold run over that list
// only; weighted values (no stage 1: every node takes part) pass no list.
template <typename V>
__global__ void k_l2_prep(int32_t* anc, V* val, V* d0, V* d1, const uint64_t* pend, int32_t* plist, uint32_t* hdr) {
  const int64_t n = hdr[3];
  bool more = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same iterations (the ballot of append_node
  // sees whole waves)
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    int32_t a = -1;
    bool part = false;
    if (i < n) {
      const int32_t pa = anc[i];
      if constexpr (!std::is_same<V, uint64_t>::value) {
        a = pa;  // weighted: no stage 1 ran, every node takes part
        part = true;
      } else if (pa <= -2) {
        a = -pa - 2;
        part = true;
      } else {
        const uint64_t w = d0[i];
        if ((w >> kL2Shift) != 0) {  // unfinished
          val[i] += w & kL2Mask;
          a = pa;
          part = true;
        }
      }
      anc[i] = a;
      d0[i] = 0;
      d1[i] = 0;
      more |= a >= 0;
    }
    if (plist) append_node(plist, &hdr[4], (int32_t)i, part);
  }
  if (more) hdr[64] = 1;
}

template <typename V>
__global__ void k_l2_round(int j, V* val, V* d0, V* d1, int32_t* a0, int32_t* a1, const int32_t* plist,
                           uint32_t* hdr) {
  if (hdr[64 + j] == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && hdr[1] == 0xFFFFFFFFu) hdr[1] = (uint32_t)(j & 1);
    return;
  }
  const int64_t m = plist ? hdr[4] : hdr[3];
  V* dc = (j & 1) ? d1 : d0;
  V* dn = (j & 1) ? d0 : d1;
  const int32_t* ac = (j & 1) ? a1 : a0;
  int32_t* an = (j & 1) ? a0 : a1;
  bool more = false;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = plist ? plist[t] : (int32_t)t;
    const int32_t a = ac[i];
    const V d = dc[i];
    if (a < 0 && d == (V)0) {  // nothing to fold or send
      an[i] = -1;
      continue;
    }
    const V v = val[i] + d;
    val[i] = v;
    dc[i] = 0;
    int32_t a2 = -1;
    if (a >= 0) {
      vadd(&dn[a], v);
      a2 = ac[a];
    }
    an[i] = a2;
    more |= a2 >= 0;
  }
  if (more) hdr[64 + j + 1] = 1;
}

// Adds the last pending increment: the resolved value of every listed node
// (the others hold theirs already).
template <typename V>
__global__ void k_l2_fold(V* val, const V* d0, const V* d1, const int32_t* plist, const uint32_t* hdr) {
  const int64_t m = plist ? hdr[4] : hdr[3];
  const V* d = (hdr[1] & 1) ? d1 : d0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = plist ? plist[t] : (int32_t)t;
    val[i] += d[i];
  }
}

// Backward: path sums H(e) = w(e) + H(parent(e)), w(e) = the receiver's
// in-tile path sum, by pointer jumping (Wyllie) over the exit slots, with two
// value and two ancestor buffers used alternately.  An exit whose ancestor
// runs out is done: its value is final in the buffer the round wrote, and it
// copies it into the other one in the next round (ancestor code -2), after
// which both hold it and the exit drops out (code -1).  The exits still in
// play are listed: workgroup w of the fixed grid keeps its own segment
// [w * seg, (w + 1) * seg) of the list of a round (L0 for even rounds, L1 for
// odd ones) with its length in cnt (cnt[w] for even rounds, cnt[G + w] for
// odd ones), so a round touches only the listed exits and appends the ones
// still in play with LDS counters (no global atomics).

// Appends v to the workgroup's segment `out` when `take`; n: LDS counter.
__device__ __forceinline__ void append_local(int32_t* out, uint32_t* n, int32_t v, bool take) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(take);
  if (m == 0) return;
  const int lane = (int)__lane_id();
  const int leader = __builtin_ctzll(m);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(n, (uint32_t)__builtin_popcountll(m));
  base = __shfl(base, leader);
  if (take) out[base + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1))] = v;
}

__global__ __launch_bounds__(256) void k_bres_init(DemTable tab, int ts, int cap, int64_t nslots,
                                                   const uint8_t* __restrict__ ex_code,
                                                   const uint16_t* __restrict__ rl, const double* __restrict__ rg,
                                                   double* b0, int32_t* a0, int32_t* L0, int64_t seg, uint32_t* cnt,
                                                   uint32_t* hdr) {
  __shared__ uint32_t ln;
  if (threadIdx.x == 0) ln = 0;
  __syncthreads();
  int32_t* mine = L0 + blockIdx.x * seg;
  bool more = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s0 = blockIdx.x * (int64_t)blockDim.x; s0 < nslots; s0 += stride) {
    const int64_t s = s0 + threadIdx.x;
    bool exit = false;
    if (s < nslots) {
      const uint8_t ec = ex_code[s];
      if (ec < 8) {
        exit = true;
        int64_t tslot;
        int32_t par;
        const bool has = exit_parent(tab, s, ts, cap, ec, rl, tslot, par);
        more |= has;
        a0[s] = has ? par : -2;
        b0[s] = rg[tslot];
      }
    }
    append_local(mine, &ln, (int32_t)s, exit);
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = ln;
  if (more) hdr[64] = 1;
}

__global__ __launch_bounds__(256) void k_bres_round(int j, double* b0, double* b1, int32_t* a0, int32_t* a1,
                                                    int32_t* L0, int32_t* L1, int64_t seg, uint32_t* cnt,
                                                    uint32_t* hdr) {
  if (hdr[64 + j] == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && hdr[2] == 0xFFFFFFFFu) hdr[2] = (uint32_t)(j & 1);
    return;
  }
  __shared__ uint32_t ln;
  if (threadIdx.x == 0) ln = 0;
  __syncthreads();
  const double* cur = (j & 1) ? b1 : b0;
  double* nxt = (j & 1) ? b0 : b1;
  const int32_t* ac = (j & 1) ? a1 : a0;
  int32_t* an = (j & 1) ? a0 : a1;
  const int64_t G = gridDim.x;
  const int32_t* Lc = ((j & 1) ? L1 : L0) + blockIdx.x * seg;
  int32_t* Ln = ((j & 1) ? L0 : L1) + blockIdx.x * seg;
  const uint32_t m = cnt[((j & 1) ? G : 0) + blockIdx.x];
  bool more = false;
  for (uint32_t t0 = 0; t0 < m; t0 += blockDim.x) {
    const uint32_t t = t0 + threadIdx.x;
    bool keep = false;
    int32_t s = 0;
    if (t < m) {
      s = Lc[t];
      const int32_t a = ac[s];
      if (a >= 0) {
        nxt[s] = cur[s] + cur[a];
        const int32_t a2 = ac[a];
        an[s] = a2 >= 0 ? a2 : -2;
        more |= a2 >= 0;
        keep = true;
      } else {  // done in the last round: copy the final value, then drop out
        nxt[s] = cur[s];
        an[s] = -1;
      }
    }
    append_local(Ln, &ln, s, keep);
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[((j & 1) ? 0 : G) + blockIdx.x] = ln;
  if (more) hdr[64 + j + 1] = 1;
}

// Records the result buffer if every round ran, and flags a cycle if
// ancestors were still left after the last round.
__global__ void k_res_finish(int rounds, int word, int nbuf, uint32_t* hdr, uint32_t* status) {
  if (hdr[word] == 0xFFFFFFFFu) {
    hdr[word] = (uint32_t)(rounds % nbuf);
    if (hdr[64 + rounds]) set_status(status, kStCycle);
  }
}

__global__ void k_zero_header(uint32_t* hdr) {
  const int i = threadIdx.x;
  if (i < (int)(kHdrBytes / 4)) hdr[i] = (i == 1 || i == 2) ? 0xFFFFFFFFu : 0u;
}

__global__ void k_clear_flags(uint32_t* hdr) {
  const int i = threadIdx.x;
  if (i < 128) hdr[64 + i] = 0;
}

// Builds the per-DEM table of a batch from the caller's device descriptors:
// one workgroup, the DEMs in chunks of 1024 with an LDS scan of the tile,
// block and super-block counts per chunk (first tile id etc. of each DEM).
__global__ __launch_bounds__(1024) void k_build_demtab(const d8_desc* __restrict__ desc, int32_t n, int ts, int bw,
                                                      int bh, DemInfo* out) {
  __shared__ int64_t sc[3][1024];
  __shared__ int64_t carry[3];
  const int tid = threadIdx.x;
  if (tid < 3) carry[tid] = 0;
  __syncthreads();
  for (int32_t c0 = 0; c0 < n; c0 += 1024) {
    const int32_t i = c0 + tid;
    DemInfo d{};
    int64_t cnt[3] = {0, 0, 0};
    if (i < n) {
      d.off = desc[i].offset;
      d.H = desc[i].rows;
      d.W = desc[i].cols;
      d.TY = (d.H + ts - 1) / ts;
      d.TX = (d.W + ts - 1) / ts;
      d.BY = (d.H + bh - 1) / bh;
      d.BX = (d.W + bw - 1) / bw;
      d.SBY = (d.H + kSuper - 1) / kSuper;
      d.SBX = (d.W + kSuper - 1) / kSuper;
      cnt[0] = (int64_t)d.TY * d.TX;
      cnt[1] = (int64_t)d.BY * d.BX;
      cnt[2] = (int64_t)d.SBY * d.SBX;
    }
    for (int k = 0; k < 3; ++k) sc[k][tid] = cnt[k];
    __syncthreads();
    // inclusive scan (Hillis-Steele) over the chunk
    for (int dlt = 1; dlt < 1024; dlt <<= 1) {
      int64_t v[3];
      for (int k = 0; k < 3; ++k) v[k] = tid >= dlt ? sc[k][tid - dlt] : 0;
      __syncthreads();
      for (int k = 0; k < 3; ++k) sc[k][tid] += v[k];
      __syncthreads();
    }
    if (i < n) {
      d.tile0 = carry[0] + sc[0][tid] - cnt[0];
      d.blk0 = carry[1] + sc[1][tid] - cnt[1];
      d.sb0 = carry[2] + sc[2][tid] - cnt[2];
      out[i] = d;
    }
    __syncthreads();
    if (tid < 3) carry[tid] += sc[tid][1023];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers --

static inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (unsigned)g;
}

hipError_t launch_zero_header(uint32_t* hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(kHdrBytes / 4), 0, s, hdr);
  return hipGetLastError();
}

hipError_t launch_build_demtab(const void* desc_dev, int32_t n, int ts, int bw, int bh, DemInfo* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_build_demtab, dim3(1), dim3(1024), 0, s, reinterpret_cast<const d8_desc*>(desc_dev), n, ts,
                     bw, bh, out);
  return hipGetLastError();
}

hipError_t launch_flowdirs(const float* dem, uint8_t* dirs, const DemTable& tab, int64_t nblocks, hipStream_t s,
                           bool steepest) {
  constexpr int RPT = kFdRows;
  if (steepest)
    hipLaunchKernelGGL((k_flowdirs<true, RPT>), dim3((unsigned)nblocks), dim3(16, 64 / RPT), 0, s, dem, dirs, tab);
  else
    hipLaunchKernelGGL((k_flowdirs<false, RPT>), dim3((unsigned)nblocks), dim3(16, 64 / RPT), 0, s, dem, dirs, tab);
  return hipGetLastError();
}

template <int BW, int BH, int TS, typename V, int CPT>
static hipError_t emit_cpt(const Plan& p, const uint8_t* dirs, const float* w, void* out, float* out_lo,
                           hipStream_t s) {
  constexpr int NT = BW * BH / CPT;
  const int64_t nb = p.span ? p.span : p.nblocks;  // a run of blocks, or all
  hipLaunchKernelGGL((k_block_emit<BW, BH, TS, V, CPT>), dim3((unsigned)nb), dim3(NT), 0, s, dirs, w, p.tab, nb,
                     p.cap, p.ex_code, p.rl, (void*)p.ex_val, out, out_lo, p.hdr, p.dem,
                     const_cast<uint8_t*>(dirs), p.span ? p.first : (int64_t)0);
  return hipGetLastError();
}

// Cells per thread of the block passes: 16, or for a 64 x 64 block of one
// tile 4, 8 or 32 (1024, 512 or 128 threads).
template <int BW, int BH, int TS, typename V>
static hipError_t emit_blk(const Plan& p, const uint8_t* dirs, const float* w, void* out, float* out_lo,
                           hipStream_t s) {
  if constexpr (BW == 64 && BH == 64) {
    if (p.cpt == 4) return emit_cpt<BW, BH, TS, V, 4>(p, dirs, w, out, out_lo, s);
    if (p.cpt == 8) return emit_cpt<BW, BH, TS, V, 8>(p, dirs, w, out, out_lo, s);
    if (p.cpt == 32) return emit_cpt<BW, BH, TS, V, 32>(p, dirs, w, out, out_lo, s);
  }
  return emit_cpt<BW, BH, TS, V, 16>(p, dirs, w, out, out_lo, s);
}

template <int TS, typename V>
static hipError_t fixup_ts(const Plan& p, const uint8_t* dirs, void* out, float* out_lo, hipStream_t s) {
  // the receiver inflows the super-block pass left in buf[2]
  const int64_t nt = p.span ? p.span : p.ntiles;  // a run of tiles, or all
  hipLaunchKernelGGL((k_fixup<TS, V>), dim3((unsigned)nt), dim3(256), 0, s, dirs, p.tab, nt, p.cap,
                     (const void*)p.buf[2], out, out_lo, p.span ? p.first : (int64_t)0);
  return hipGetLastError();
}

// Launch shape of the tile passes.  Tile 64: one 64 x 64 tile per workgroup
// of 64 * waves threads, waves 2, 4, 8 (default) or 16, i.e. 32, 16, 8 or 4
// cells per thread (counts also take the walk pass, waves 1, 2, 4).  Tile 32:
// workgroups of waves = 1 (default), 2 or 4 tiles, 16 cells per thread.
// Tile 128 (counts): one tile per workgroup of 1024 threads (waves 16).
void count_block_dims(int ts, int waves, int& bw, int& bh) {
  if (ts == 32) {
    bw = waves >= 2 ? 64 : 32;
    bh = waves >= 4 ? 64 : 32;
  } else {
    bw = ts;
    bh = ts;
  }
}

bool waves_ok(int ts, int waves, bool counts) {
  if (waves == 0) return true;
  if (ts == 32) return waves == 1 || waves == 2 || waves == 4;
  if (ts == 64) return waves == 2 || waves == 4 || waves == 8 || waves == 16 || (counts && waves == 1);
  if (ts == 128) return counts && waves == 16;
  return false;
}

template <typename V>
static hipError_t tile_pass(const Plan& p, const uint8_t* dirs, const float* w, bool final_pass, void* out,
                            float* out_lo, hipStream_t s) {
  constexpr bool kCount = std::is_same<V, uint32_t>::value;
  if (final_pass) {
    switch (p.ts) {
      case 32: return fixup_ts<32, V>(p, dirs, out, out_lo, s);
      case 64: return fixup_ts<64, V>(p, dirs, out, out_lo, s);
      case 128:
        if constexpr (kCount) return fixup_ts<128, V>(p, dirs, out, out_lo, s);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (kCount)
    if (p.ts == 64 && !p.dem && p.wpt > 0) return launch_walk_count(p, dirs, static_cast<uint32_t*>(out), p.wpt, s);
  if (p.ts == 32 && p.bw == 32 && p.bh == 32) return emit_blk<32, 32, 32, V>(p, dirs, w, out, out_lo, s);
  if (p.ts == 32 && p.bw == 64 && p.bh == 32) return emit_blk<64, 32, 32, V>(p, dirs, w, out, out_lo, s);
  if (p.ts == 32 && p.bw == 64 && p.bh == 64) return emit_blk<64, 64, 32, V>(p, dirs, w, out, out_lo, s);
  if (p.ts == 64) return emit_blk<64, 64, 64, V>(p, dirs, w, out, out_lo, s);
  if constexpr (kCount)
    if (p.ts == 128) return emit_blk<128, 128, 128, V>(p, dirs, w, out, out_lo, s);
  return hipErrorInvalidValue;
}

hipError_t launch_count_tiles(const Plan& p, const uint8_t* dirs, bool final_pass, uint32_t* out, hipStream_t s) {
  return tile_pass<uint32_t>(p, dirs, nullptr, final_pass, out, nullptr, s);
}

hipError_t launch_weighted_tiles(const Plan& p, const uint8_t* dirs, const float* w, bool final_pass, float* out,
                                 float* out_lo, hipStream_t s) {
  return tile_pass<double>(p, dirs, w, final_pass, out, out_lo, s);
}

template <int BW, int BH, int TS, int CPT>
static hipError_t bwd_cpt(const Plan& p, const uint8_t* dirs, const float* g, bool fin, float* out, hipStream_t s) {
  constexpr int NT = BW * BH / CPT;
  const double* b0 = reinterpret_cast<const double*>(p.buf[0]);
  const double* b1 = reinterpret_cast<const double*>(p.buf[1]);
  double* ev = reinterpret_cast<double*>(p.ex_val);
  if (fin)
    hipLaunchKernelGGL((k_bwd_final<BW, BH, TS>), dim3((unsigned)p.nblocks), dim3(256), 0, s, p.tab, p.nblocks, p.cap,
                       p.blo, p.broot, b0, b1, p.hdr, out);
  else
    hipLaunchKernelGGL((k_block_bwd<BW, BH, TS, CPT>), dim3((unsigned)p.nblocks), dim3(NT), 0, s, dirs, g, p.tab,
                       p.nblocks, p.cap, p.ex_code, p.rl, ev, p.blo, p.broot, out, p.hdr);
  return hipGetLastError();
}

template <int BW, int BH, int TS>
static hipError_t bwd_blk(const Plan& p, const uint8_t* dirs, const float* g, bool fin, float* out, hipStream_t s) {
  if constexpr (BW == 64 && BH == 64) {
    if (p.cpt == 4) return bwd_cpt<BW, BH, TS, 4>(p, dirs, g, fin, out, s);
    if (p.cpt == 8) return bwd_cpt<BW, BH, TS, 8>(p, dirs, g, fin, out, s);
    if (p.cpt == 32) return bwd_cpt<BW, BH, TS, 32>(p, dirs, g, fin, out, s);
  }
  return bwd_cpt<BW, BH, TS, 16>(p, dirs, g, fin, out, s);
}

hipError_t launch_backward_tiles(const Plan& p, const uint8_t* dirs, const float* g, bool final_pass, float* out,
                                 hipStream_t s) {
  if (p.ts == 32 && p.bw == 32 && p.bh == 32) return bwd_blk<32, 32, 32>(p, dirs, g, final_pass, out, s);
  if (p.ts == 32 && p.bw == 64 && p.bh == 32) return bwd_blk<64, 32, 32>(p, dirs, g, final_pass, out, s);
  if (p.ts == 32 && p.bw == 64 && p.bh == 64) return bwd_blk<64, 64, 32>(p, dirs, g, final_pass, out, s);
  if (p.ts == 64) return bwd_blk<64, 64, 64>(p, dirs, g, final_pass, out, s);
  return hipErrorInvalidValue;
}

template <int TS, typename LV, typename V, bool DOWN>
static void group_launch(const Plan& p, hipStream_t s) {
  V* ev = reinterpret_cast<V*>(p.ex_val);
  V* b0 = reinterpret_cast<V*>(p.buf[0]);
  V* b1 = reinterpret_cast<V*>(p.buf[1]);
  uint64_t* b2 = p.buf[2];
  hipLaunchKernelGGL((k_group<TS, LV, V, DOWN>), dim3((unsigned)p.nsb), dim3(GroupDims<TS, LV>::NT), 0, s, p.tab,
                     p.nsb, p.ex_code,
                     p.rl, ev, b0, p.anc[1], p.anc[0], b1, b2, b0, reinterpret_cast<V*>(b2), p.hdr, p.hdr);
}

template <typename LV, typename V, bool DOWN>
static void group_pass(const Plan& p, hipStream_t s) {
  switch (p.ts) {
    case 32: group_launch<32, LV, V, DOWN>(p, s); break;
    case 64: group_launch<64, LV, V, DOWN>(p, s); break;
    default: group_launch<128, LV, V, DOWN>(p, s); break;
  }
}

template <typename LV, typename V>
static hipError_t fres(const Plan& p, hipStream_t s) {
  V* b0 = reinterpret_cast<V*>(p.buf[0]);
  V* b1 = reinterpret_cast<V*>(p.buf[1]);
  V* b2 = reinterpret_cast<V*>(p.buf[2]);
  // Nodes: at most one per super-block perimeter cell.  One thread per node
  // for the walks (their work is a chain of dependent random accesses); the
  // other passes loop over the nodes with a grid of one resident wave of
  // workgroups (2048 x 256 threads fill the GPU), so a round with nothing
  // left to do costs one small dispatch.
  const int64_t maxn = std::min<int64_t>(p.nslots, p.nsb * 4 * kSuper);
  const unsigned gn = (unsigned)std::max<int64_t>(1, (maxn + 255) / 256);
  const unsigned g = (unsigned)std::min<int64_t>(gn, 2048);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(128), 0, s, p.hdr);
  group_pass<LV, V, false>(p, s);
  uint64_t* pend = p.buf[2];
  hipLaunchKernelGGL(k_l2_init, dim3(g), dim3(256), 0, s, p.anc[1], p.anc[0], p.hdr);
  // Counts only: the weighted stage 1 would need a fence between its two
  // atomics (an L2 write-back on this GPU) per step; doubling does it all.
  if constexpr (std::is_same<V, uint64_t>::value)
    hipLaunchKernelGGL((k_l2_walk<V>), dim3(gn), dim3(256), 0, s, p.anc[0], b0, b1, pend, p.hdr);
  int32_t* pl = std::is_same<V, uint64_t>::value ? p.plist : nullptr;
  hipLaunchKernelGGL((k_l2_prep<V>), dim3(g), dim3(256), 0, s, p.anc[0], b0, b1, b2, pend, pl, p.hdr);
  // a forest of at most maxn nodes is done after floor(log2(maxn)) + 1
  // doubling rounds; flags still set after them mean a cycle
  int rounds = 1;
  while (((int64_t)1 << (rounds - 1)) <= maxn && rounds < kMaxRounds) ++rounds;
  rounds = std::min(rounds, p.rounds);
  for (int j = 0; j < rounds; ++j)
    hipLaunchKernelGGL((k_l2_round<V>), dim3(g), dim3(256), 0, s, j, b0, b1, b2, p.anc[0], p.list, pl, p.hdr);
  hipLaunchKernelGGL(k_res_finish, dim3(1), dim3(1), 0, s, rounds, 1, 2, p.hdr, p.hdr);
  hipLaunchKernelGGL((k_l2_fold<V>), dim3(g), dim3(256), 0, s, b0, b1, b2, pl, p.hdr);
  group_pass<LV, V, true>(p, s);
  return hipGetLastError();
}

hipError_t launch_forward_resolve(const Plan& p, bool weighted, hipStream_t s) {
  return weighted ? fres<double, double>(p, s) : fres<uint32_t, uint64_t>(p, s);
}

hipError_t launch_backward_resolve(const Plan& p, hipStream_t s) {
  double* b0 = reinterpret_cast<double*>(p.buf[0]);
  double* b1 = reinterpret_cast<double*>(p.buf[1]);
  const double* rg = reinterpret_cast<const double*>(p.ex_val);
  // the same workgroups for the init and every round, each with its own
  // segment of the exit lists (list_grid, as the layout sized them)
  const unsigned gr = (unsigned)std::max<int64_t>(1, list_grid(p.nslots));
  const int64_t seg = list_segment(p.nslots, gr);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(128), 0, s, p.hdr);
  hipLaunchKernelGGL(k_bres_init, dim3(gr), dim3(256), 0, s, p.tab, p.ts, p.cap, p.nslots, p.ex_code, p.rl, rg, b0,
                     p.anc[0], p.list, seg, p.lcnt, p.hdr);
  for (int j = 0; j < p.rounds; ++j)
    hipLaunchKernelGGL(k_bres_round, dim3(gr), dim3(256), 0, s, j, b0, b1, p.anc[0], p.anc[1], p.list, p.plist, seg,
                       p.lcnt, p.hdr);
  hipLaunchKernelGGL(k_res_finish, dim3(1), dim3(1), 0, s, p.rounds, 2, 2, p.hdr, p.hdr);
  return hipGetLastError();
}

}  // namespace d8
