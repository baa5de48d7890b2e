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
#include <type_traits>

#include "d8_internal.hpp"
#include "d8.h"

namespace d8 {

constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr uint64_t kPendOne = 1ull << 40;

// ------------------------------------------------------------------ flowdirs --
// D8 "lowest of eight" (Sec. 1): a 16x16-thread block covers a 64x64-cell
// tile; each thread owns a 4x4 patch and reads its 6x6 neighbourhood.
constexpr int kFdTile = 64;

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

__global__ __launch_bounds__(256) void k_flowdirs(const float* __restrict__ dem, uint8_t* __restrict__ dirs,
                                                   DemTable tab) {
  const int64_t tile = blockIdx.x;
  const DemInfo dm = dem_of_tile(tab, tile);
  const int64_t lt = tile - dm.tile0;
  const int64_t ty = lt / dm.TX, tx = lt - ty * dm.TX;
  const int64_t H = dm.H, W = dm.W;
  const float* z = dem + dm.off;
  uint8_t* d = dirs + dm.off;
  const int64_t y0 = ty * kFdTile + 4 * threadIdx.y;
  const int64_t x0 = tx * kFdTile + 4 * threadIdx.x;
  if (y0 >= H || x0 >= W) return;
  float v[6][6];
#pragma unroll
  for (int rr = 0; rr < 6; ++rr) {
    const int64_t yy = y0 - 1 + rr;
    const bool rin = yy >= 0 && yy < H;
#pragma unroll
    for (int cc = 0; cc < 6; ++cc) {
      const int64_t xx = x0 - 1 + cc;
      v[rr][cc] = (rin && xx >= 0 && xx < W) ? z[yy * W + xx] : 0.0f;
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
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
        k = nanadj ? kNone : lowest8(c, n0, n1, n2, n3, n4, n5, n6, n7);
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

// ----------------------------------------------------------- tile helpers --

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin
// (block b runs on XCD b % 8); give each XCD a contiguous run of tiles so that
// neighbouring tiles, which share cache lines of the direction field, meet in
// the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t n) {
  const int64_t q = n >> 3, rem = n & 7;
  const int64_t x = bid & 7, i = bid >> 3;
  return x * q + (x < rem ? x : rem) + i;
}

struct TileGeo {
  DemInfo dm;
  int64_t tile, y0, x0;
  int tw, th;
};

__device__ __forceinline__ TileGeo tile_geo(const DemTable& tab, int64_t tile, int ts) {
  TileGeo g;
  g.tile = tile;
  g.dm = dem_of_tile(tab, tile);
  const int64_t lt = tile - g.dm.tile0;
  const int64_t ty = lt / g.dm.TX, tx = lt - ty * g.dm.TX;
  g.y0 = ty * ts;
  g.x0 = tx * ts;
  g.th = (int)min((int64_t)ts, (int64_t)g.dm.H - g.y0);
  g.tw = (int)min((int64_t)ts, (int64_t)g.dm.W - g.x0);
  return g;
}

// Global slot id of the perimeter cell at global (gy, gx) of the DEM dm.
__device__ __forceinline__ int64_t slot_of_cell(const DemInfo& dm, int64_t gy, int64_t gx, int ts, int cap) {
  const int64_t nty = gy / ts, ntx = gx / ts;
  const int64_t ntile = dm.tile0 + nty * dm.TX + ntx;
  const int nth = (int)min((int64_t)ts, (int64_t)dm.H - nty * ts);
  const int ntw = (int)min((int64_t)ts, (int64_t)dm.W - ntx * ts);
  return ntile * cap + perim_slot((int)(gy - nty * ts), (int)(gx - ntx * ts), ntw, nth);
}

// Stage the tile's direction codes with a one-cell halo into LDS.  When the
// tile's rows are 4-byte aligned (full-width tile, width and offset multiples
// of 4) the (TS+2) rows are fetched as 32-bit words, all loads of a thread
// issued before any is consumed; the two halo columns are single bytes.
template <int TS>
__device__ __forceinline__ void load_codes(uint8_t* code, const uint8_t* __restrict__ dirs, const TileGeo& g) {
  constexpr int HS = TS + 2;
  constexpr int WPR = TS / 4;     // 32-bit words per tile row
  constexpr int NW = HS * WPR;    // rows y0-1 .. y0+TS
  constexpr int MAXW = 9;         // >= ceil(NW / 64) for TS <= 32, ceil(NW / 256) for TS <= 64 ...
  const uint8_t* D = dirs + g.dm.off;
  const int64_t H = g.dm.H, W = g.dm.W;
  const int NT = blockDim.x, tid = threadIdx.x;
  const bool vec = g.tw == TS && (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(D + g.x0) & 3) == 0) &&
                   (NW + NT - 1) / NT <= MAXW && 2 * HS <= 2 * NT;
  if (vec) {
    uint32_t v[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
      const int i = tid + k * NT;
      v[k] = 0xFEFEFEFEu;  // kOutside bytes
      if (i < NW) {
        const int lr = i / WPR, q = i - lr * WPR;
        const int64_t gy = g.y0 + lr - 1;
        if (gy >= 0 && gy < H) v[k] = *reinterpret_cast<const uint32_t*>(D + gy * W + g.x0 + 4 * q);
      }
    }
    // halo columns x0-1 and x0+TS (2*HS bytes; at most two per thread)
    uint8_t hb[2] = {kOutside, kOutside};
    int hidx[2] = {-1, -1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = tid + k * NT;
      if (i < 2 * HS) {
        const int lr = i >> 1, side = i & 1;
        const int64_t gy = g.y0 + lr - 1, gx = side ? g.x0 + TS : g.x0 - 1;
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
    if (hidx[0] >= 0) code[hidx[0]] = hb[0];
    if (hidx[1] >= 0) code[hidx[1]] = hb[1];
  } else {
    for (int i = tid; i < HS * HS; i += NT) {
      const int lr = i / HS, lc = i - lr * HS;
      const int64_t gy = g.y0 + lr - 1, gx = g.x0 + lc - 1;
      uint8_t v = kOutside;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = D[gy * W + gx];
      code[i] = v;
    }
  }
}

// Validated code of in-tile cell (r, c): 0..7 (drains to a valid cell), 8
// (outlet, or an invalid code / target, which also raises the status word).
template <int TS>
__device__ __forceinline__ uint8_t eff_code(const uint8_t* code, int r, int c, const TileGeo& g,
                                            uint32_t* status) {
  constexpr int HS = TS + 2;
  const uint8_t k = code[(r + 1) * HS + c + 1];
  if (k == kNone) return kNone;
  if (k > kNone) {
    set_status(status, kStBadDir);
    return kNone;
  }
  const int tr = r + ddr(k), tc = c + ddc(k);
  const int64_t gy = g.y0 + tr, gx = g.x0 + tc;
  if (gy < 0 || gy >= g.dm.H || gx < 0 || gx >= g.dm.W || code[(tr + 1) * HS + tc + 1] == kNoData) {
    set_status(status, kStBadDir);
    return kNone;
  }
  return k;
}

// In-tile input count and mask, and the mask of inputs from outside the tile.
template <int TS>
__device__ __forceinline__ void inputs_of(const uint8_t* code, int r, int c, const TileGeo& g, int& pend,
                                          uint32_t& inm, uint32_t& ext) {
  constexpr int HS = TS + 2;
  pend = 0;
  inm = 0;
  ext = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int nr = r + ddr(i), nc = c + ddc(i);
    if (code[(nr + 1) * HS + nc + 1] == ((i + 4) & 7)) {
      if (nr >= 0 && nr < g.th && nc >= 0 && nc < g.tw) {
        ++pend;
        inm |= 1u << i;
      } else {
        ext |= 1u << i;
      }
    }
  }
}

template <int TS>
__device__ __forceinline__ uint32_t ext_mask(const uint8_t* code, int r, int c, const TileGeo& g) {
  int p;
  uint32_t m, e;
  inputs_of<TS>(code, r, c, g, p, m, e);
  return e;
}

// Sum of the resolved areas of the exits (in other tiles) that drain into
// receiver (r, c): the inflow the paper's master returns for a receiver.
template <typename V>
__device__ __forceinline__ V gather_inflow(const V* __restrict__ F, uint32_t ext, int r, int c, const TileGeo& g,
                                           int ts, int cap) {
  V x = 0;
  for (int i = 0; i < 8; ++i) {
    if (ext & (1u << i)) {
      const int64_t gy = g.y0 + r + ddr(i), gx = g.x0 + c + ddc(i);
      x += F[slot_of_cell(g.dm, gy, gx, ts, cap)];
    }
  }
  return x;
}

// --------------------------------------------- counts: push-style tile walk --
// LDS state per cell, one word: value | pending inputs (4 bits) | in-tile
// target (or kTgtExit: drains to another tile, kTgtEnd: outlet).  A walker
// carries the final value v of its cell to the target with one LDS atomic that
// adds v and retires one pending input; the arrival that retires the last
// input owns the target and continues downstream (Alg. 2's tail recursion).
// Integer sums: the result does not depend on the arrival order.
template <typename Wd, int TS>
struct CountWord {
  static constexpr int kCells = TS * TS;
  static constexpr int TB = (kCells <= 256 ? 9 : kCells <= 1024 ? 11 : kCells <= 4096 ? 13 : 15);
  static constexpr int PB = 4;
  static constexpr int VB = (int)sizeof(Wd) * 8 - TB - PB;
  static constexpr Wd VMASK = (Wd(1) << VB) - 1;
  static constexpr Wd PONE = Wd(1) << VB;
  static constexpr int TSH = VB + PB;
  static constexpr uint32_t kTgtExit = kCells;
  static constexpr uint32_t kTgtEnd = kCells + 1;
  __device__ static Wd make(uint32_t tgt, Wd val) { return val | (Wd(tgt) << TSH); }
  __device__ static uint32_t tgt(Wd w) { return (uint32_t)(w >> TSH); }
  __device__ static uint32_t pend(Wd w) { return (uint32_t)(w >> VB) & 15u; }
  __device__ static Wd val(Wd w) { return w & VMASK; }
};

// Word type of the count walk: 32 bits while the largest tile-local value
// (TS*TS, emit pass) fits, else 64 bits (final pass: values up to 2^32-1).
template <int TS, bool FINAL>
using CountW = typename std::conditional<(!FINAL && TS <= 64), uint32_t, unsigned long long>::type;

template <int TS, bool FINAL>
struct CountSmem {
  CountW<TS, FINAL> st[TS * TS];
  uint8_t code[(TS + 2) * (TS + 2)];
};

template <int TS, int NT, bool FINAL>
__global__ __launch_bounds__(NT) void k_tile_count(const uint8_t* __restrict__ dirs, DemTable tab, int64_t ntiles,
                                                   int cap, uint8_t* __restrict__ ex_code,
                                                   uint16_t* __restrict__ rl, uint64_t* __restrict__ ex_val,
                                                   const uint64_t* __restrict__ F0, const uint64_t* __restrict__ F1,
                                                   const uint64_t* __restrict__ F2, const uint32_t* __restrict__ hdr,
                                                   uint32_t* __restrict__ out, uint32_t* __restrict__ status) {
  using Wd = CountW<TS, FINAL>;
  using CW = CountWord<Wd, TS>;
  constexpr int CPT = TS * TS / NT;
  static_assert(CPT * NT == TS * TS && CPT <= 32, "cells per thread");
  __shared__ CountSmem<TS, FINAL> sm;
  constexpr int HS = TS + 2;
  const TileGeo g = tile_geo(tab, xcd_tile(blockIdx.x, ntiles), TS);
  const int tid = threadIdx.x;
  load_codes<TS>(sm.code, dirs, g);
  __syncthreads();

  const uint64_t* F = nullptr;
  if (FINAL) {
    const uint32_t fi = hdr[1];
    F = fi == 0 ? F0 : (fi == 1 ? F1 : F2);
  }
  // Phase A: per own cell, target and initial value.
  uint32_t tg[CPT];
  uint32_t valid = 0;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    const int r = c / TS, col = c % TS;
    tg[k] = CW::kTgtEnd;
    Wd word = CW::make(CW::kTgtEnd, 0);
    if (r < g.th && col < g.tw && sm.code[(r + 1) * HS + col + 1] != kNoData) {
      valid |= 1u << k;
      const uint8_t e = eff_code<TS>(sm.code, r, col, g, status);
      if (e < 8) {
        const int tr = r + ddr(e), tc = col + ddc(e);
        tg[k] = (tr >= 0 && tr < g.th && tc >= 0 && tc < g.tw) ? (uint32_t)(tr * TS + tc) : CW::kTgtExit;
      }
      Wd v = 1;
      if (FINAL && on_perim(r, col, g.tw, g.th)) {
        const uint32_t ext = ext_mask<TS>(sm.code, r, col, g);
        if (ext) v += (Wd)gather_inflow<uint64_t>(F, ext, r, col, g, TS, cap);
      }
      word = CW::make(tg[k], v);
    }
    sm.st[c] = word;
  }
  __syncthreads();
  // Phase B: count in-tile inputs (Alg. 1) by one atomic increment per edge.
#pragma unroll
  for (int k = 0; k < CPT; ++k)
    if (tg[k] < (uint32_t)(TS * TS)) atomicAdd(&sm.st[tg[k]], CW::PONE);
  __syncthreads();
  uint32_t src = 0;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = tid + k * NT;
    if ((valid >> k) & 1u) {
      if (CW::pend(sm.st[c]) == 0) src |= 1u << k;
    }
  }
  // Every wave must read its sources before any walker starts retiring
  // inputs (a retired cell would otherwise look like a source).
  __syncthreads();

  // Walk: one step per iteration for every lane that has work.
  uint32_t t = CW::kTgtEnd;
  Wd v = 0;
  for (;;) {
    if (t >= (uint32_t)(TS * TS)) {
      if (src == 0) break;
      const int k = __builtin_ctz(src);
      src &= src - 1;
      const Wd w = sm.st[tid + k * NT];
      v = CW::val(w);
      t = CW::tgt(w);
      continue;
    }
    const Wd old = atomicAdd(&sm.st[t], (Wd)(v - CW::PONE));
    if (CW::pend(old) == 1) {
      v += CW::val(old);
      t = CW::tgt(old);
    } else {
      t = CW::kTgtEnd;
    }
  }
  __syncthreads();

  // Any cell still waiting for an input lies on or below a cycle.
  bool cyc = false;
#pragma unroll
  for (int k = 0; k < CPT; ++k)
    if (CW::pend(sm.st[tid + k * NT])) cyc = true;
  if (cyc) set_status(status, kStCycle);

  if (FINAL) {
    uint32_t* O = out + g.dm.off;
    const int64_t W = g.dm.W;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int c = tid + k * NT;
      const int r = c / TS, col = c % TS;
      if (r < g.th && col < g.tw) O[(g.y0 + r) * W + g.x0 + col] = (uint32_t)CW::val(sm.st[c]);
    }
  } else {
    const int P = perim_count(g.tw, g.th);
    const int64_t sb = g.tile * cap;
    for (int j = tid; j < cap; j += NT) {
      uint8_t ec = 0xFF;
      if (j < P) {
        int r, col;
        perim_cell(j, g.tw, g.th, r, col);
        const int c = r * TS + col;
        const Wd w = sm.st[c];
        if (CW::tgt(w) == CW::kTgtExit) {
          ec = sm.code[(r + 1) * HS + col + 1];
          ex_val[sb + j] = (uint64_t)CW::val(w);
        }
        if (sm.code[(r + 1) * HS + col + 1] != kNoData && ext_mask<TS>(sm.code, r, col, g)) {
          // Receiver: follow its in-tile path to the exit it leaves by.
          int u = c, steps = 0;
          uint16_t link = 0xFFFF;
          for (;;) {
            const uint32_t tt = CW::tgt(sm.st[u]);
            if (tt == CW::kTgtExit) {
              link = (uint16_t)perim_slot(u / TS, u % TS, g.tw, g.th);
              break;
            }
            if (tt == CW::kTgtEnd) break;
            u = (int)tt;
            if (++steps > TS * TS) {
              set_status(status, kStCycle);
              break;
            }
          }
          rl[sb + j] = link;
        }
      }
      ex_code[sb + j] = ec;
    }
  }
}

// ------------------------------------------ weighted: gather-style tile walk --
// Values are float32 pairs (hi, lo).  The arrival that retires a cell's last
// pending input sums the cell as w (+ resolved inflow) + the inputs' values in
// the fixed order E..SE, so the result does not depend on arrival order.
template <int TS>
struct WSmem {
  df val[TS * TS];
  uint32_t pend[TS * TS / 4];  // one byte per cell
  uint8_t cv[TS * TS];         // validated code
  uint8_t inm[TS * TS];        // in-tile input mask
  uint8_t code[(TS + 2) * (TS + 2)];
};

__device__ __forceinline__ int noff(int i, int ts) { return ddr(i) * ts + ddc(i); }

template <int TS, bool FINAL>
__global__ __launch_bounds__(1024) void k_tile_weighted(const uint8_t* __restrict__ dirs,
                                                        const float* __restrict__ wts, DemTable tab, int64_t ntiles,
                                                        int cap, uint8_t* __restrict__ ex_code,
                                                        uint16_t* __restrict__ rl, double* __restrict__ ex_val,
                                                        const double* __restrict__ F0, const double* __restrict__ F1,
                                                        const double* __restrict__ F2,
                                                        const uint32_t* __restrict__ hdr, float* __restrict__ out,
                                                        float* __restrict__ out_lo, uint32_t* __restrict__ status) {
  __shared__ WSmem<TS> sm;
  constexpr int HS = TS + 2;
  const TileGeo g = tile_geo(tab, xcd_tile(blockIdx.x, ntiles), TS);
  const int NT = blockDim.x, tid = threadIdx.x;
  const int cpt = (TS * TS + NT - 1) / NT;
  load_codes<TS>(sm.code, dirs, g);
  __syncthreads();
  const double* F = nullptr;
  if (FINAL) {
    const uint32_t fi = hdr[1];
    F = fi == 0 ? F0 : (fi == 1 ? F1 : F2);
  }
  const float* Wp = wts ? wts + g.dm.off : nullptr;
  const int64_t W = g.dm.W;
  uint8_t* pendb = reinterpret_cast<uint8_t*>(sm.pend);
  uint64_t src = 0;
  for (int k = 0; k < cpt; ++k) {
    const int c = tid + k * NT;
    if (c >= TS * TS) break;
    const int r = c / TS, col = c % TS;
    df v = {0.0f, 0.0f};
    uint8_t e = kNoData, m = 0, p = 0;
    if (r < g.th && col < g.tw && sm.code[(r + 1) * HS + col + 1] != kNoData) {
      e = eff_code<TS>(sm.code, r, col, g, status);
      int pend;
      uint32_t inm, ext;
      inputs_of<TS>(sm.code, r, col, g, pend, inm, ext);
      v.hi = Wp ? Wp[(g.y0 + r) * W + g.x0 + col] : 1.0f;
      if (FINAL && ext) v = df_add(v, df_from_double(gather_inflow<double>(F, ext, r, col, g, TS, cap)));
      m = (uint8_t)inm;
      p = (uint8_t)pend;
      if (pend == 0) src |= 1ull << k;
    }
    sm.val[c] = v;
    sm.cv[c] = e;
    sm.inm[c] = m;
    pendb[c] = p;
  }
  __syncthreads();

  int cur = -1;
  for (;;) {
    if (cur < 0) {
      if (src == 0) break;
      const int k = __builtin_ctzll(src);
      src &= src - 1;
      cur = tid + k * NT;
    }
    int nxt = -1;
    const uint32_t e = sm.cv[cur];
    if (e < 8) {
      const int r = cur / TS, col = cur % TS;
      const int tr = r + ddr(e), tc = col + ddc(e);
      if (tr >= 0 && tr < g.th && tc >= 0 && tc < g.tw) {
        const int t = tr * TS + tc;
        const uint32_t sh = 8 * (t & 3);
        const uint32_t old = __hip_atomic_fetch_add(&sm.pend[t >> 2], (uint32_t)(0u - (1u << sh)), __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        if (((old >> sh) & 0xFF) == 1) {
          df a = sm.val[t];
          const uint32_t m = sm.inm[t];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (m & (1u << i)) a = df_add(a, sm.val[t + noff(i, TS)]);
          sm.val[t] = a;
          nxt = t;
        }
      }
    }
    cur = nxt;
  }
  __syncthreads();

  bool cyc = false;
  for (int k = 0; k < cpt; ++k) {
    const int c = tid + k * NT;
    if (c >= TS * TS) break;
    if (pendb[c] != 0) cyc = true;
  }
  if (cyc) set_status(status, kStCycle);

  if (FINAL) {
    float* O = out + g.dm.off;
    float* OL = out_lo ? out_lo + g.dm.off : nullptr;
    for (int k = 0; k < cpt; ++k) {
      const int c = tid + k * NT;
      if (c >= TS * TS) break;
      const int r = c / TS, col = c % TS;
      if (r < g.th && col < g.tw) {
        const df a = sm.val[c];
        const float s = a.hi + a.lo;
        O[(g.y0 + r) * W + g.x0 + col] = s;
        if (OL) OL[(g.y0 + r) * W + g.x0 + col] = (a.hi - s) + a.lo;
      }
    }
  } else {
    const int P = perim_count(g.tw, g.th);
    const int64_t sb = g.tile * cap;
    for (int j = tid; j < cap; j += NT) {
      uint8_t ec = 0xFF;
      if (j < P) {
        int r, col;
        perim_cell(j, g.tw, g.th, r, col);
        const uint32_t k = sm.cv[r * TS + col];
        if (k < 8) {
          const int tr = r + ddr(k), tc = col + ddc(k);
          if (!(tr >= 0 && tr < g.th && tc >= 0 && tc < g.tw)) {
            ec = (uint8_t)k;
            ex_val[sb + j] = df_to_double(sm.val[r * TS + col]);
          }
        }
        if (k != kNoData && ext_mask<TS>(sm.code, r, col, g)) {
          int ur = r, uc = col, steps = 0;
          uint16_t link = 0xFFFF;
          for (;;) {
            const uint32_t k2 = sm.cv[ur * TS + uc];
            if (k2 >= 8) break;
            const int tr = ur + ddr(k2), tc = uc + ddc(k2);
            if (tr < 0 || tr >= g.th || tc < 0 || tc >= g.tw) {
              link = (uint16_t)perim_slot(ur, uc, g.tw, g.th);
              break;
            }
            ur = tr;
            uc = tc;
            if (++steps > g.tw * g.th) {
              set_status(status, kStCycle);
              break;
            }
          }
          rl[sb + j] = link;
        }
      }
      ex_code[sb + j] = ec;
    }
  }
}

// --------------------------------------------- backward: in-tile path sums --
// G(c) = g(c) + G(target(c)).  Inside a tile this is a path sum to the tile's
// root, computed by pointer jumping (each round doubles the covered path
// length); S, the pointer and the root label are updated through registers
// between barriers.  Deterministic.
constexpr uint16_t kEnd = 0xFFFF;
constexpr int kBwdMaxCpt = 16;

template <int TS>
struct BSmem {
  df S[TS * TS];
  uint16_t ptr[TS * TS];
  uint16_t lab[TS * TS];
  uint8_t cv[TS * TS];
  uint8_t code[(TS + 2) * (TS + 2)];
};

template <int TS, bool FINAL>
__global__ __launch_bounds__(1024) void k_tile_backward(const uint8_t* __restrict__ dirs,
                                                        const float* __restrict__ gin, DemTable tab, int64_t ntiles,
                                                        int cap, uint8_t* __restrict__ ex_code,
                                                        uint16_t* __restrict__ rl, double* __restrict__ rg,
                                                        const double* __restrict__ H0, const double* __restrict__ H1,
                                                        const uint32_t* __restrict__ hdr, float* __restrict__ out,
                                                        uint32_t* __restrict__ status) {
  __shared__ BSmem<TS> sm;
  constexpr int HS = TS + 2;
  const TileGeo g = tile_geo(tab, xcd_tile(blockIdx.x, ntiles), TS);
  const int NT = blockDim.x, tid = threadIdx.x;
  const int cpt = (TS * TS + NT - 1) / NT;
  load_codes<TS>(sm.code, dirs, g);
  __syncthreads();
  const float* G = gin + g.dm.off;
  const int64_t W = g.dm.W;
  for (int k = 0; k < cpt; ++k) {
    const int c = tid + k * NT;
    if (c >= TS * TS) break;
    const int r = c / TS, col = c % TS;
    df s = {0.0f, 0.0f};
    uint16_t p = kEnd, lb = kEnd;
    uint8_t e = kNoData;
    if (r < g.th && col < g.tw && sm.code[(r + 1) * HS + col + 1] != kNoData) {
      e = eff_code<TS>(sm.code, r, col, g, status);
      s.hi = G[(g.y0 + r) * W + g.x0 + col];
      lb = (uint16_t)c;
      if (e < 8) {
        const int tr = r + ddr(e), tc = col + ddc(e);
        if (tr >= 0 && tr < g.th && tc >= 0 && tc < g.tw) {
          p = (uint16_t)(tr * TS + tc);
          lb = kEnd;
        }
      }
    }
    sm.S[c] = s;
    sm.ptr[c] = p;
    sm.lab[c] = lb;
    sm.cv[c] = e;
  }
  __syncthreads();

  const int lim = TS * TS * 2;  // a cycle never converges; stop after enough rounds
  for (int round = 0;; ++round) {
    df ns[kBwdMaxCpt];
    uint16_t np[kBwdMaxCpt], nl[kBwdMaxCpt];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kBwdMaxCpt; ++k) {
      const int c = tid + k * NT;
      np[k] = kEnd;
      if (k < cpt && c < TS * TS) {
        const uint16_t p = sm.ptr[c];
        if (p != kEnd) {
          ns[k] = df_add(sm.S[c], sm.S[p]);
          np[k] = sm.ptr[p];
          nl[k] = sm.lab[p];
          any = true;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBwdMaxCpt; ++k) {
      const int c = tid + k * NT;
      if (k < cpt && c < TS * TS && sm.ptr[c] != kEnd) {
        sm.S[c] = ns[k];
        sm.ptr[c] = np[k];
        sm.lab[c] = nl[k];
      }
    }
    if (!__syncthreads_or(any)) break;
    if ((1 << min(round, 30)) > lim) {
      set_status(status, kStCycle);
      break;
    }
  }
  __syncthreads();

  if (FINAL) {
    const uint32_t fi = hdr[2];
    const double* Hb = fi == 0 ? H0 : H1;
    float* O = out + g.dm.off;
    const int64_t sb = g.tile * cap;
    for (int k = 0; k < cpt; ++k) {
      const int c = tid + k * NT;
      if (c >= TS * TS) break;
      const int r = c / TS, col = c % TS;
      if (r < g.th && col < g.tw) {
        double acc = df_to_double(sm.S[c]);
        const uint16_t root = sm.lab[c];
        if (sm.cv[c] != kNoData && root != kEnd && sm.cv[root] < 8) {
          acc += Hb[sb + perim_slot(root / TS, root % TS, g.tw, g.th)];
        }
        O[(g.y0 + r) * W + g.x0 + col] = (float)acc;
      }
    }
  } else {
    const int P = perim_count(g.tw, g.th);
    const int64_t sb = g.tile * cap;
    for (int j = tid; j < cap; j += NT) {
      uint8_t ec = 0xFF;
      if (j < P) {
        int r, col;
        perim_cell(j, g.tw, g.th, r, col);
        const int c = r * TS + col;
        const uint32_t k = sm.cv[c];
        if (k < 8) {
          const int tr = r + ddr(k), tc = col + ddc(k);
          if (!(tr >= 0 && tr < g.th && tc >= 0 && tc < g.tw)) ec = (uint8_t)k;
        }
        if (k != kNoData && ext_mask<TS>(sm.code, r, col, g)) {
          const uint16_t root = sm.lab[c];
          uint16_t link = 0xFFFF;
          if (root != kEnd && sm.cv[root] < 8) link = (uint16_t)perim_slot(root / TS, root % TS, g.tw, g.th);
          rl[sb + j] = link;
          rg[sb + j] = df_to_double(sm.S[c]);
        }
      }
      ex_code[sb + j] = ec;
    }
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

// Forward: subtree sums F = (I - P)^-1 L over the exit forest by doubling,
// F = (I + P)(I + P^2)(I + P^4)... L, where P^(2^j) adds a node's value into
// its 2^j-th ancestor.  Three rotating value buffers (read / accumulate /
// clear) and two ancestor buffers; round j stops early once no ancestors are
// left, and records which buffer holds the result.
template <typename V>
__global__ void k_fres_init(DemTable tab, int ts, int cap, int64_t nslots, const uint8_t* __restrict__ ex_code,
                            const uint16_t* __restrict__ rl, const V* __restrict__ ex_val, V* b0, V* b1, int32_t* a0,
                            uint32_t* hdr) {
  bool more = false;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t ec = ex_code[s];
    if (ec >= 8) continue;
    int64_t ts_;
    int32_t par;
    more |= exit_parent(tab, s, ts, cap, ec, rl, ts_, par);
    a0[s] = par;
    b0[s] = ex_val[s];
    b1[s] = 0;
  }
  if (more) hdr[64] = 1;
}

template <typename V>
__global__ void k_fres_round(int j, int64_t nslots, const uint8_t* __restrict__ ex_code, V* b0, V* b1, V* b2,
                             int32_t* a0, int32_t* a1, uint32_t* hdr) {
  if (hdr[64 + j] == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && hdr[1] == 0xFFFFFFFFu) hdr[1] = (uint32_t)(j % 3);
    return;
  }
  V* bufs[3] = {b0, b1, b2};
  const V* cur = bufs[j % 3];
  V* nxt = bufs[(j + 1) % 3];
  V* clr = bufs[(j + 2) % 3];
  const int32_t* ac = (j & 1) ? a1 : a0;
  int32_t* an = (j & 1) ? a0 : a1;
  bool more = false;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    if (ex_code[s] >= 8) continue;
    const V v = cur[s];
    vadd(&nxt[s], v);
    const int32_t a = ac[s];
    int32_t a2 = -1;
    if (a >= 0) {
      vadd(&nxt[a], v);
      a2 = ac[a];
    }
    an[s] = a2;
    clr[s] = 0;
    more |= a2 >= 0;
  }
  if (more) hdr[64 + j + 1] = 1;
}

// Backward: path sums H(e) = w(e) + H(parent(e)), w(e) = the receiver's
// in-tile path sum, by pointer jumping (Wyllie).  Two buffers each.
__global__ void k_bres_init(DemTable tab, int ts, int cap, int64_t nslots, const uint8_t* __restrict__ ex_code,
                            const uint16_t* __restrict__ rl, const double* __restrict__ rg, double* b0, int32_t* a0,
                            uint32_t* hdr) {
  bool more = false;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t ec = ex_code[s];
    if (ec >= 8) continue;
    int64_t tslot;
    int32_t par;
    more |= exit_parent(tab, s, ts, cap, ec, rl, tslot, par);
    a0[s] = par;
    b0[s] = rg[tslot];
  }
  if (more) hdr[64] = 1;
}

__global__ void k_bres_round(int j, int64_t nslots, const uint8_t* __restrict__ ex_code, double* b0, double* b1,
                             int32_t* a0, int32_t* a1, uint32_t* hdr) {
  if (hdr[64 + j] == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && hdr[2] == 0xFFFFFFFFu) hdr[2] = (uint32_t)(j & 1);
    return;
  }
  const double* cur = (j & 1) ? b1 : b0;
  double* nxt = (j & 1) ? b0 : b1;
  const int32_t* ac = (j & 1) ? a1 : a0;
  int32_t* an = (j & 1) ? a0 : a1;
  bool more = false;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * blockDim.x) {
    if (ex_code[s] >= 8) continue;
    const int32_t a = ac[s];
    if (a >= 0) {
      nxt[s] = cur[s] + cur[a];
      const int32_t a2 = ac[a];
      an[s] = a2;
      more |= a2 >= 0;
    } else {
      nxt[s] = cur[s];
      an[s] = -1;
    }
  }
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

// Builds the per-DEM table of a batch from the caller's device descriptors
// (a serial prefix over the DEMs; n is small).
__global__ void k_build_demtab(const d8_desc* __restrict__ desc, int32_t n, int ts, DemInfo* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t t0 = 0;
  for (int32_t i = 0; i < n; ++i) {
    DemInfo d;
    d.off = desc[i].offset;
    d.H = desc[i].rows;
    d.W = desc[i].cols;
    d.TY = (d.H + ts - 1) / ts;
    d.TX = (d.W + ts - 1) / ts;
    d.tile0 = t0;
    t0 += (int64_t)d.TY * d.TX;
    out[i] = d;
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

hipError_t launch_build_demtab(const void* desc_dev, int32_t n, int ts, DemInfo* out, hipStream_t s) {
  hipLaunchKernelGGL(k_build_demtab, dim3(1), dim3(64), 0, s, reinterpret_cast<const d8_desc*>(desc_dev), n, ts,
                     out);
  return hipGetLastError();
}

hipError_t launch_flowdirs(const float* dem, uint8_t* dirs, const DemTable& tab, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_flowdirs, dim3((unsigned)nblocks), dim3(16, 16), 0, s, dem, dirs, tab);
  return hipGetLastError();
}

template <int TS, int NT>
static hipError_t count_ts(const Plan& p, const uint8_t* dirs, bool fin, uint32_t* out, hipStream_t s) {
  uint32_t* st = p.hdr;
  const uint64_t* b0 = p.buf[0];
  const uint64_t* b1 = p.buf[1];
  const uint64_t* b2 = p.buf[2];
  if (fin)
    hipLaunchKernelGGL((k_tile_count<TS, NT, true>), dim3((unsigned)p.ntiles), dim3(NT), 0, s, dirs, p.tab, p.ntiles,
                       p.cap, p.ex_code, p.rl, p.ex_val, b0, b1, b2, p.hdr, out, st);
  else
    hipLaunchKernelGGL((k_tile_count<TS, NT, false>), dim3((unsigned)p.ntiles), dim3(NT), 0, s, dirs, p.tab,
                       p.ntiles, p.cap, p.ex_code, p.rl, p.ex_val, b0, b1, b2, p.hdr, out, st);
  return hipGetLastError();
}

hipError_t launch_count_tiles(const Plan& p, const uint8_t* dirs, bool final_pass, uint32_t* out, int nt,
                              hipStream_t s) {
  switch (p.ts) {
    case 32:
      if (nt <= 64) return count_ts<32, 64>(p, dirs, final_pass, out, s);
      if (nt <= 128) return count_ts<32, 128>(p, dirs, final_pass, out, s);
      return count_ts<32, 256>(p, dirs, final_pass, out, s);
    case 64:
      if (nt <= 128) return count_ts<64, 128>(p, dirs, final_pass, out, s);
      if (nt <= 256) return count_ts<64, 256>(p, dirs, final_pass, out, s);
      return count_ts<64, 512>(p, dirs, final_pass, out, s);
    case 128:
      if (nt <= 512) return count_ts<128, 512>(p, dirs, final_pass, out, s);
      return count_ts<128, 1024>(p, dirs, final_pass, out, s);
  }
  return hipErrorInvalidValue;
}

template <int TS>
static hipError_t weighted_ts(const Plan& p, const uint8_t* dirs, const float* w, bool fin, float* out,
                              float* out_lo, int nt, hipStream_t s) {
  const double* b0 = reinterpret_cast<const double*>(p.buf[0]);
  const double* b1 = reinterpret_cast<const double*>(p.buf[1]);
  const double* b2 = reinterpret_cast<const double*>(p.buf[2]);
  double* ev = reinterpret_cast<double*>(p.ex_val);
  if (fin)
    hipLaunchKernelGGL((k_tile_weighted<TS, true>), dim3((unsigned)p.ntiles), dim3(nt), 0, s, dirs, w, p.tab,
                       p.ntiles, p.cap, p.ex_code, p.rl, ev, b0, b1, b2, p.hdr, out, out_lo, p.hdr);
  else
    hipLaunchKernelGGL((k_tile_weighted<TS, false>), dim3((unsigned)p.ntiles), dim3(nt), 0, s, dirs, w, p.tab,
                       p.ntiles, p.cap, p.ex_code, p.rl, ev, b0, b1, b2, p.hdr, out, out_lo, p.hdr);
  return hipGetLastError();
}

hipError_t launch_weighted_tiles(const Plan& p, const uint8_t* dirs, const float* w, bool final_pass, float* out,
                                 float* out_lo, int nt, hipStream_t s) {
  switch (p.ts) {
    case 32: return weighted_ts<32>(p, dirs, w, final_pass, out, out_lo, nt, s);
    case 64: return weighted_ts<64>(p, dirs, w, final_pass, out, out_lo, nt, s);
  }
  return hipErrorInvalidValue;
}

template <int TS>
static hipError_t backward_ts(const Plan& p, const uint8_t* dirs, const float* g, bool fin, float* out, int nt,
                              hipStream_t s) {
  const double* b0 = reinterpret_cast<const double*>(p.buf[0]);
  const double* b1 = reinterpret_cast<const double*>(p.buf[1]);
  double* ev = reinterpret_cast<double*>(p.ex_val);
  if (fin)
    hipLaunchKernelGGL((k_tile_backward<TS, true>), dim3((unsigned)p.ntiles), dim3(nt), 0, s, dirs, g, p.tab,
                       p.ntiles, p.cap, p.ex_code, p.rl, ev, b0, b1, p.hdr, out, p.hdr);
  else
    hipLaunchKernelGGL((k_tile_backward<TS, false>), dim3((unsigned)p.ntiles), dim3(nt), 0, s, dirs, g, p.tab,
                       p.ntiles, p.cap, p.ex_code, p.rl, ev, b0, b1, p.hdr, out, p.hdr);
  return hipGetLastError();
}

hipError_t launch_backward_tiles(const Plan& p, const uint8_t* dirs, const float* g, bool final_pass, float* out,
                                 int nt, hipStream_t s) {
  switch (p.ts) {
    case 32: return backward_ts<32>(p, dirs, g, final_pass, out, nt, s);
    case 64: return backward_ts<64>(p, dirs, g, final_pass, out, nt, s);
  }
  return hipErrorInvalidValue;
}

template <typename V>
static hipError_t fres(const Plan& p, hipStream_t s) {
  V* b0 = reinterpret_cast<V*>(p.buf[0]);
  V* b1 = reinterpret_cast<V*>(p.buf[1]);
  V* b2 = reinterpret_cast<V*>(p.buf[2]);
  const V* ev = reinterpret_cast<const V*>(p.ex_val);
  const unsigned g = grid_for(p.nslots, 256);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(128), 0, s, p.hdr);
  hipLaunchKernelGGL((k_fres_init<V>), dim3(g), dim3(256), 0, s, p.tab, p.ts, p.cap, p.nslots, p.ex_code, p.rl, ev,
                     b0, b1, p.anc[0], p.hdr);
  for (int j = 0; j < p.rounds; ++j)
    hipLaunchKernelGGL((k_fres_round<V>), dim3(g), dim3(256), 0, s, j, p.nslots, p.ex_code, b0, b1, b2, p.anc[0],
                       p.anc[1], p.hdr);
  hipLaunchKernelGGL(k_res_finish, dim3(1), dim3(1), 0, s, p.rounds, 1, 3, p.hdr, p.hdr);
  return hipGetLastError();
}

hipError_t launch_forward_resolve(const Plan& p, bool weighted, hipStream_t s) {
  return weighted ? fres<double>(p, s) : fres<uint64_t>(p, s);
}

hipError_t launch_backward_resolve(const Plan& p, hipStream_t s) {
  double* b0 = reinterpret_cast<double*>(p.buf[0]);
  double* b1 = reinterpret_cast<double*>(p.buf[1]);
  const double* rg = reinterpret_cast<const double*>(p.ex_val);
  const unsigned g = grid_for(p.nslots, 256);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(128), 0, s, p.hdr);
  hipLaunchKernelGGL(k_bres_init, dim3(g), dim3(256), 0, s, p.tab, p.ts, p.cap, p.nslots, p.ex_code, p.rl, rg, b0,
                     p.anc[0], p.hdr);
  for (int j = 0; j < p.rounds; ++j)
    hipLaunchKernelGGL(k_bres_round, dim3(g), dim3(256), 0, s, j, p.nslots, p.ex_code, b0, b1, p.anc[0], p.anc[1],
                       p.hdr);
  hipLaunchKernelGGL(k_res_finish, dim3(1), dim3(1), 0, s, p.rounds, 2, 2, p.hdr, p.hdr);
  return hipGetLastError();
}

}  // namespace d8
