// Counts tile pass by last-arriver walks, one wave per 64 x 64 tile.
//
// Alg. 2 of Barnes, Lehman & Mulla (PDPTA 2011) evaluates a part's internal
// up-slope area from a queue of cells whose inputs are all known: a cell is
// taken, its area is added to the cell it drains into, and that cell enters
// the queue once its last input has arrived.  Here each lane of the wave runs
// that loop for one walk at a time: it starts at a cell with no in-tile input
// (a source), delivers the area it carries to the target with one LDS atomic
// that also retires one pending input of the target, and carries on with the
// target only if its own delivery was the last one (the tail recursion of
// Alg. 2).  Inflows from other tiles are the unknowns of Sec. 3 and are left
// out (Alg. 3), so the pass yields each tile's local areas, the partial area of
// every exit and, for every receiver, the exit its in-tile path leaves by
// (Alg. 4's Cell_V / Origin links).
//
// LDS word of a cell (one per cell, plus a border ring):
//   bits  0..12  A - 1 so far (sum of the areas delivered by its inputs)
//   bits 16..19  in-tile inputs still to deliver
//   bits 24..31  signed offset, in words, to the cell it drains into (0: none)
// A walk's delivery adds (area - 1 << 16): the pending field never borrows,
// since every input delivers exactly once.  Cells draining out of the tile
// point into the border ring, whose words have no offset, so walks end there.
// Rows are stored south to north so the three north-going offsets are
// positive: byte tables indexed by the D8 code (v_perm_b32) then give 0 for
// code 8, whose selector picks the sign of table byte 1.
#include <algorithm>
#include <type_traits>

#include "d8_internal.hpp"
#include "d8.h"

namespace d8 {

// Optional per-phase cycle stamps for measurement builds (D8_WALK_STAMPS):
// the cycles each workgroup spends between consecutive stamps are summed into
// workspace header words 800.. (64-bit), iteration counts into words 840...
#ifdef D8_WALK_STAMPS
#define WSTAMP(i) wts_[i] = __builtin_amdgcn_s_memtime()
#else
#define WSTAMP(i)
#endif

namespace wk {
constexpr int T = 64;                // tile side
constexpr int S = 68;                // LDS words per row (16-byte aligned rows)
constexpr int NW = S * (T + 2) + 4;  // rows -1..64, plus the east border of row -1
constexpr int QCAP = 1984;           // source queue entries per phase
constexpr int QLEN = QCAP + 64;      // + one discard slot per lane
constexpr int RCAP = 4 * T;          // receiver entries (>= 4T - 4)
constexpr int HW = T + 2;            // halo row length (columns -1..64)
constexpr uint32_t kPOne = 1u << 16;
constexpr uint32_t kPMask = 0xFu << 16;
constexpr uint32_t kAccMask = 0xFFFu;
constexpr uint32_t kBorder = 0x8000u;  // set in border-ring words only
// Byte tables (byte k = value for code k): signed word offsets E, NE, N, NW,
// W, SW, S, SE; and 1 for a cell that drains somewhere.
constexpr uint32_t kOffLo = 0x01u | (uint32_t)(uint8_t)(S + 1) << 8 | (uint32_t)(uint8_t)S << 16 |
                            (uint32_t)(uint8_t)(S - 1) << 24;
constexpr uint32_t kOffHi = 0xFFu | (uint32_t)(uint8_t)(-S - 1) << 8 | (uint32_t)(uint8_t)(-S) << 16 |
                            (uint32_t)(uint8_t)(-S + 1) << 24;
constexpr uint32_t kHasLo = 0x01010101u, kHasHi = 0x01010101u;

// Word index of tile cell (r, c), r and c in -1..64.  (r, 64) shares its word
// with (r - 1, -4); columns -3 and -2 are padding no walk reaches.
__device__ __forceinline__ int widx(int r, int c) { return (T - r) * S + c + 4; }

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Bytes of w that are >= 9 (D8 codes outside 0..8: NoData, beyond the DEM,
// or invalid): 0x80 in each such byte.
__device__ __forceinline__ uint32_t high_bytes(uint32_t w) {
  return (((w & 0x7F7F7F7Fu) + 0x77777777u) | w) & 0x80808080u;
}

// Workgroup barrier that orders LDS only: it waits for this wave's LDS
// operations, not for its global stores (a full __syncthreads would wait for
// the previous tile's output stores to reach memory).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Exclusive prefix sum of x over the NT threads of the workgroup (waves of
// 64), and the total.  sc: NT / 64 words of LDS scratch.
template <int NT>
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t* sc, uint32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t v = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  if (lane == 63) sc[wv] = v;
  lds_barrier();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t s = sc[w];
    before += w < wv ? s : 0u;
    tot += s;
  }
  lds_barrier();
  total = tot;
  return before + v - x;
}
}  // namespace wk

__device__ __forceinline__ uint32_t lds_add_rtn(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Codes of one tile as the walk pass holds them in registers: for each
// 16-cell row chunk of the thread, four 4-cell words (254 beyond the DEM).
// Row chunk k of thread tid is chunk m = k * NT + tid: row m / 4, columns
// 16 (m % 4) .. +15.
template <int RPT>
struct TileCodes {
  uint4 c[RPT];
  uint8_t h[5];  // halo: top (column lane), bottom, west (row lane), east, corner
};

template <int NT, int RPT>
__device__ __forceinline__ void load_codes(TileCodes<RPT>& tc, const uint8_t* __restrict__ dirs, const TileGeo& g) {
  using namespace wk;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t W = g.dm.W, H = g.dm.H;
  const uint8_t* D = dirs + g.dm.off;
  const bool full = g.tw == T && g.th == T && (W & 15) == 0 && ((reinterpret_cast<uintptr_t>(D) & 15) == 0);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int m = k * NT + tid, r = m >> 2, c0 = 16 * (m & 3);
    if (full) {
      tc.c[k] = *reinterpret_cast<const uint4*>(D + (g.y0 + r) * W + g.x0 + c0);
    } else {
      uint32_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int c = c0 + 4 * q + b;
          const uint32_t x =
              (r < g.th && c < g.tw) ? (uint32_t)D[(g.y0 + r) * W + g.x0 + c] : (uint32_t)kOutside;
          v[q] |= x << (8 * b);
        }
      }
      tc.c[k] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  }
  if (tid < 64) {
    auto at = [&](int64_t gy, int64_t gx) -> uint8_t {
      return (gy >= 0 && gy < H && gx >= 0 && gx < W) ? D[gy * W + gx] : kOutside;
    };
    const int64_t x0 = g.x0, y0 = g.y0;
    tc.h[0] = at(y0 - 1, x0 + lane);
    tc.h[1] = at(y0 + g.th, x0 + lane);
    tc.h[2] = at(y0 + lane, x0 - 1);
    tc.h[3] = at(y0 + lane, x0 + g.tw);
    const int64_t yy = (lane & 1) ? y0 + g.th : y0 - 1, xx = (lane & 2) ? x0 + T : x0 - 1;
    tc.h[4] = lane < 4 ? at(yy, xx) : (uint8_t)kOutside;
  }
}

// Persistent: each workgroup takes tiles from the counter of its XCD (tiles
// of one XCD form a contiguous band, so the halo rows a tile reads sit in the
// same L2 as its neighbours'), and loads the next tile's codes while it walks
// the current one.  WPT waves share a tile and take the source queue in
// interleaved blocks of 64 entries.
// Resident waves per SIMD when seven workgroups share a CU (the LDS limit).
template <int WPT>
struct WalkOcc {
  static constexpr int kWavesPerSimd = (7 * WPT + 3) / 4;
};

template <int WPT>
__global__ __launch_bounds__(64 * WPT) __attribute__((amdgpu_waves_per_eu(WalkOcc<WPT>::kWavesPerSimd))) void k_walk_count(const uint8_t* __restrict__ dirs, DemTable tab,
                                                         int64_t ntiles, int cap, uint8_t* __restrict__ ex_code,
                                                         uint16_t* __restrict__ rl, uint64_t* __restrict__ ex_val,
                                                         uint32_t* __restrict__ out, uint32_t* __restrict__ status,
                                                         int64_t first, uint32_t* __restrict__ ctr) {
  using namespace wk;
  constexpr int NT = 64 * WPT;
  constexpr int RPT = 4 / WPT;                    // 16-cell row chunks per thread
  constexpr int NPS = (4 * T - 4 + NT - 1) / NT;  // perimeter slots per thread
  __shared__ __attribute__((aligned(16))) uint32_t wd[NW];
  __shared__ __attribute__((aligned(16))) uint16_t q[QLEN];
  __shared__ uint16_t rend[RCAP];  // receiver walks: word index of the exit left by, or 0xFFFF
  __shared__ uint8_t rq[RCAP];     // receivers' perimeter slots
  __shared__ uint32_t cnt[8];      // [0] next tile, [2] receivers, [4..] scan scratch, [7] slow flag
  // codes around the tile (top, bottom: columns -1..64; west, east: rows),
  // kept in the queue's space until the queue is filled
  uint8_t* halo = reinterpret_cast<uint8_t*>(q);
  // exit code of every perimeter slot (0xFF: not an exit), in the padding
  // words (columns -3, -2) of LDS rows 0..31
  auto pex = [&](int j) -> uint8_t& { return reinterpret_cast<uint8_t*>(&wd[(j >> 3) * S + 1])[j & 7]; };
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // this XCD's band of tiles and counter
  const int xcd = blockIdx.x & 7;
  const int64_t band0 = xcd_tile(xcd, ntiles) - 0, band1 = xcd == 7 ? ntiles : xcd_tile(xcd + 1, ntiles);
  auto grab = [&]() -> int64_t {
    const uint32_t k = atomicAdd(&ctr[xcd], 1u);
    return band0 + k < band1 ? band0 + (int64_t)k : (int64_t)-1;
  };
  if (tid < 8) cnt[tid] = tid == 0 ? (uint32_t)grab() : 0u;
  lds_barrier();
  int64_t cur = (int32_t)cnt[0];
  lds_barrier();  // every thread has read cnt[0] before it is reused
  TileCodes<RPT> tc;
  TileGeo g{};
  if (cur >= 0) {
    g = tile_geo(tab, first + cur, T);
    load_codes<NT, RPT>(tc, dirs, g);
  }
  bool cyc = false, wait_in = false, badd = false;
  while (cur >= 0) {
#ifdef D8_WALK_STAMPS
    uint64_t wts_[10] = {};
    uint32_t nbulk_ = 0, ntail_ = 0;
#endif
    WSTAMP(0);
    // next tile id (read after the tile's first barrier)
    if (tid == 0) cnt[0] = (uint32_t)grab();
    const int64_t W = g.dm.W;
    const int tw = g.tw, th = g.th;
    if (tid < 64) {
      halo[lane + 1] = tc.h[0];
      halo[HW + lane + 1] = tc.h[1];
      halo[2 * HW + lane] = tc.h[2];
      halo[3 * HW + lane] = tc.h[3];
      if (lane < 4) halo[(lane & 1) * HW + ((lane & 2) ? HW - 1 : 0)] = tc.h[4];
    }
    // Tiles holding codes >= 9 (NoData, cells beyond the DEM, invalid codes)
    // take them as outlets for the walks; invalid ones set the status word.
    uint32_t anyhi = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      anyhi |= high_bytes(tc.c[k].x) | high_bytes(tc.c[k].y) | high_bytes(tc.c[k].z) | high_bytes(tc.c[k].w);
    if (anyhi) cnt[7] = 1u;
    lds_barrier();
    const int64_t nxt = (int32_t)cnt[0];
    const bool slow = cnt[7] != 0u;
    uint32_t s4[RPT][4];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const uint32_t cw[4] = {tc.c[k].x, tc.c[k].y, tc.c[k].z, tc.c[k].w};
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        s4[k][qq] = cw[qq];
        if (slow) {
          const uint32_t c = cw[qq];
          const uint32_t h = high_bytes(c);
          const uint32_t fe = ((c & 0x7F7F7F7Fu) + 0x02020202u) & c & 0x80808080u;  // bytes 254, 255
          badd |= (h & ~fe) != 0u;
          const uint32_t m = h | (h - (h >> 7));  // 0xFF in each byte >= 9
          s4[k][qq] = (c & ~m) | (0x08080808u & m);
        }
      }
    }
    WSTAMP(1);
    // ---- LDS words: border ring kBorder, cells (offset << 24)
    {
      uint4* w4 = reinterpret_cast<uint4*>(wd);
      const uint4 z = make_uint4(kBorder, kBorder, kBorder, kBorder);
      // row 64 (LDS row 0) and row -1 (LDS row T+1): 17 vectors each; columns
      // -4..-1 of rows 0..63: one vector each; the last 4 words.
      for (int v = tid; v < 2 * (S / 4) + T + 1; v += NT) {
        int wi;
        if (v < S / 4) wi = 4 * v;
        else if (v < 2 * (S / 4)) wi = (T + 1) * S + 4 * (v - S / 4);
        else if (v < 2 * (S / 4) + T) wi = (v - 2 * (S / 4) + 1) * S;
        else wi = (T + 2) * S;
        w4[wi / 4] = z;
      }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int m = k * NT + tid, r = m >> 2, c0 = 16 * (m & 3);
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const uint32_t o4 = perm(kOffHi, kOffLo, s4[k][qq]);
        uint4 v;
        v.x = perm(o4, 0u, 0x040C0C0Cu);
        v.y = perm(o4, 0u, 0x050C0C0Cu);
        v.z = perm(o4, 0u, 0x060C0C0Cu);
        v.w = perm(o4, 0u, 0x070C0C0Cu);
        *reinterpret_cast<uint4*>(&wd[widx(r, c0 + 4 * qq)]) = v;
      }
    }
    lds_barrier();
    WSTAMP(2);
    // ---- pending inputs: every cell that drains somewhere adds one to its
    // target's count (cells draining out of the tile count into the border).
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int m = k * NT + tid, r = m >> 2, c0 = 16 * (m & 3);
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const uint32_t o4 = perm(kOffHi, kOffLo, s4[k][qq]);
        const uint32_t h4 = perm(kHasHi, kHasLo, s4[k][qq]);
        const int w0 = widx(r, c0 + 4 * qq);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int off = (int)(int8_t)(uint8_t)(o4 >> (8 * b));
          const uint32_t v = perm(0u, h4, 0x0C000C0Cu | ((uint32_t)b << 16));
          __hip_atomic_fetch_add(&wd[w0 + b + off], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    // ---- the next tile's codes load while this one is walked
    TileCodes<RPT> tn;
    TileGeo gn{};
    if (nxt >= 0) {
      gn = tile_geo(tab, first + nxt, T);
      load_codes<NT, RPT>(tn, dirs, gn);
    }
    WSTAMP(3);

    // ---- perimeter: receivers (fed from outside the tile) and exits (draining
    // into a valid cell of another tile), from the halo
    const int np = perim_count(tw, th);
    auto hcode = [&](int nr, int nc) -> uint32_t {
      if (nr < 0) return halo[nc + 1];
      if (nr >= th) return halo[HW + nc + 1];
      if (nc < 0) return halo[2 * HW + nr];
      return halo[3 * HW + nr];
    };
    {
      uint32_t mine = 0;
      bool isr[NPS];
#pragma unroll
      for (int sI = 0; sI < NPS; ++sI) {
        const int j = tid + NT * sI;
        isr[sI] = false;
        if (j < np) {
          int lr, lc;
          perim_cell(j, tw, th, lr, lc);
          bool rcv = false;
#pragma unroll
          for (int d = 0; d < 8; ++d) {
            const int nr = lr + ddr_t(d), nc = lc + ddc_t(d);
            if (nr < 0 || nr >= th || nc < 0 || nc >= tw) rcv |= hcode(nr, nc) == (uint32_t)((d + 4) & 7);
          }
          isr[sI] = rcv;
          // exit: the word's offset tells where the cell drains (0: nowhere)
          const uint32_t w = wd[widx(lr, lc)];
          uint8_t ec = 0xFF;
          const int off = (int)w >> 24;
          if (off != 0) {
            // the code whose offset this is (offsets are distinct)
            uint32_t d = 0;
#pragma unroll
            for (int dd = 1; dd < 8; ++dd) d = (off == (int)(int8_t)(uint8_t)(kOffLo >> (8 * (dd & 3))) && dd < 4) ||
                                                     (dd >= 4 && off == (int)(int8_t)(uint8_t)(kOffHi >> (8 * (dd - 4))))
                                                 ? (uint32_t)dd : d;
            const int nr = lr + ddr_t(d), nc = lc + ddc_t(d);
            if (nr < 0 || nr >= th || nc < 0 || nc >= tw) {
              const uint32_t tcode = hcode(nr, nc);
              if (tcode == kOutside || tcode == kNoData) badd = true;  // off the grid or into NoData
              else ec = (uint8_t)d;
            }
          }
          pex(j) = ec;
        }
        mine += isr[sI];
      }
      uint32_t nrq;
      uint32_t pos = block_scan<NT>(mine, &cnt[4], nrq);
#pragma unroll
      for (int sI = 0; sI < NPS; ++sI)
        if (isr[sI]) rq[pos++] = (uint8_t)(tid + NT * sI);
      if (tid == 0) cnt[2] = nrq;
    }

    // ---- sources: cells with no pending input that drain somewhere.  The
    // queue holds the word index of each source's target (its first delivery).
    uint64_t sb = 0;  // source bits: 16 per row chunk
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int m = k * NT + tid, r = m >> 2, c0 = 16 * (m & 3);
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const uint4 v = *reinterpret_cast<const uint4*>(&wd[widx(r, c0 + 4 * qq)]);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        const uint32_t c = qq == 0 ? tc.c[k].x : qq == 1 ? tc.c[k].y : qq == 2 ? tc.c[k].z : tc.c[k].w;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const bool src = (w[b] & kPMask) == 0u && w[b] >= 0x01000000u;
          sb |= (uint64_t)src << (16 * k + 4 * qq + b);
          if (slow && ((c >> (8 * b)) & 0xFFu) == kNoData && (w[b] & kPMask) != 0u)
            badd = true;  // a cell drains into NoData
        }
      }
    }
    uint32_t ntot;
    (void)block_scan<NT>((uint32_t)__builtin_popcountll(sb), &cnt[4], ntot);
    const uint32_t nrq = cnt[2];
    // One phase when the queue holds every source; else four phases over
    // quarters of the cells (at most 1024 each).
    const int nphase = ntot <= (uint32_t)QCAP ? 1 : 4;
    for (int ph = 0; ph < nphase; ++ph) {
      // phase ph takes a quarter of each thread's cells (4 RPT source bits)
      const uint64_t qm = (4 * RPT >= 64) ? ~0ull : ((1ull << (4 * RPT)) - 1ull);
      const uint64_t sbp = nphase == 1 ? sb : sb & (qm << (4 * RPT * ph));
      uint32_t nq;
      uint32_t pos = block_scan<NT>((uint32_t)__builtin_popcountll(sbp), &cnt[4], nq);
      // every cell of a group with a source writes an entry: sources at the
      // next queue position, the others into the lane's discard slot
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int m = k * NT + tid, r = m >> 2, c0 = 16 * (m & 3);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const uint32_t f = (uint32_t)(sbp >> (16 * k + 4 * qq)) & 15u;
          if (f == 0u) continue;
          const uint32_t o4 = perm(kOffHi, kOffLo, s4[k][qq]);
          const int w0 = widx(r, c0 + 4 * qq);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int off = (int)(int8_t)(uint8_t)(o4 >> (8 * b));
            const uint32_t bit = (f >> b) & 1u;
            q[bit ? pos : (uint32_t)(QCAP + lane)] = (uint16_t)(w0 + b + off);
            pos += bit;
          }
        }
      }
      lds_barrier();
      WSTAMP(4);
      const bool last_phase = ph == nphase - 1;

      // ---- the walks.  t: word index of the next delivery; dlt: what it
      // adds, (area carried) - (one pending input).  Bulk loop: accumulation
      // walks fed from the queue, each lane prefetching its next entry.
      auto qslot = [&](uint32_t n) -> uint32_t { return ((n >> 6) * WPT + wv) * 64 + (n & 63); };
      uint32_t qc = 64;  // this wave's next entry number to hand out
      uint32_t myslot = qslot(lane);
      uint32_t pe = q[myslot < (uint32_t)QLEN ? myslot : QLEN - 1];
      uint32_t t = 0u, dlt = 0u;
      bool act = false;
      for (;;) {
        const bool has = myslot < nq;
        if (__ballot(has) == 0u) break;  // every entry of this wave handed out
#ifdef D8_WALK_STAMPS
        ++nbulk_;
#endif
        const bool take = !act && has;
        const uint64_t tm = __ballot(take);
        const uint32_t nslot = qslot(qc + lane_rank(tm));
        t = take ? pe : t;
        dlt = take ? 1u - kPOne : dlt;
        myslot = take ? nslot : myslot;
        act = act || take;
        qc += (uint32_t)__builtin_popcountll(tm);
        pe = q[myslot < (uint32_t)QLEN ? myslot : QLEN - 1];
        if (act) {
          const uint32_t old = lds_add_rtn(&wd[t], dlt);
          act = (old & kPMask) == kPOne && old >= 0x01000000u;  // last delivery, and a target
          dlt += (old & kAccMask) + 1u;
          t += (uint32_t)((int)old >> 24);
        }
      }
      WSTAMP(5);
      // Tail loop: the remaining accumulation walks, and the receiver walks of
      // the last phase (read-only: they deliver 0 and always continue; rid and
      // prev track the receiver and the cell before the current one).
      uint32_t pmask = kPMask, pone = kPOne, amask = kAccMask, one = 1u;
      uint32_t prev = 0u;
      int rid = -1;
      uint32_t rh = last_phase ? 0u : nrq;  // receivers of this wave (k % WPT == wv) handed out
      for (int it = 0;; ++it) {
        if (rh * WPT + wv < nrq) {
          const bool want = !act;
          const uint64_t rm = __ballot(want);
          const uint32_t slot = (rh + lane_rank(rm)) * WPT + wv;
          if (want && slot < nrq) {
            int lr, lc;
            perim_cell((int)rq[slot], tw, th, lr, lc);
            rid = (int)slot;
            t = (uint32_t)widx(lr, lc);
            dlt = 0u;
            pmask = 0u;
            pone = 0u;
            amask = 0u;
            one = 0u;
            act = true;
          }
          rh += (uint32_t)__builtin_popcountll(rm);
        }
        if (!__any(act)) break;
#ifdef D8_WALK_STAMPS
        ++ntail_;
#endif
        if (it > 64 * T * T) {  // only a cycle keeps a receiver walk going
          cyc = true;
          break;
        }
        if (act) {
          const uint32_t old = lds_add_rtn(&wd[t], dlt);
          const bool cont = (old & pmask) == pone && old >= 0x01000000u;
          dlt += (old & amask) + one;
          if (rid >= 0 && !cont) {
            // a receiver walk ends: in the border ring the previous cell is
            // the exit it leaves by; at a cell without target there is none
            rend[rid] = (old & kBorder) ? (uint16_t)prev : (uint16_t)0xFFFFu;
            rid = -1;
          }
          prev = t;
          t += (uint32_t)((int)old >> 24);
          act = cont;
        }
      }
      lds_barrier();
    }
    WSTAMP(6);

    // ---- tile-local areas (16 lanes per tile row, 16 bytes each); a cell
    // still waiting for an input lies on a cycle
    {
      uint32_t* O = out + g.dm.off + g.y0 * W + g.x0;
      const bool full = tw == T && th == T && (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(O) & 15) == 0);
      const int rr = tid >> 4, cq = (tid & 15) * 4;
#pragma unroll
      for (int i = 0; i < 16 / WPT; ++i) {
        const int r = 4 * WPT * i + rr;
        const uint4 v = *reinterpret_cast<const uint4*>(&wd[widx(r, cq)]);
        uint32_t a[4] = {(v.x & kAccMask) + 1u, (v.y & kAccMask) + 1u, (v.z & kAccMask) + 1u,
                         (v.w & kAccMask) + 1u};
        if (!slow && full) {
          wait_in |= ((v.x | v.y | v.z | v.w) & kPMask) != 0u;
          *reinterpret_cast<uint4*>(O + r * W + cq) = make_uint4(a[0], a[1], a[2], a[3]);
        } else if (!slow) {
          wait_in |= ((v.x | v.y | v.z | v.w) & kPMask) != 0u;
#pragma unroll
          for (int b = 0; b < 4; ++b) O[r * W + cq + b] = a[b];
        } else {
          // codes again for NoData / beyond-the-DEM cells (they output 0)
          const uint32_t wv4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const bool in = r < th && cq + b < tw;
            const uint32_t c = in ? (uint32_t)dirs[g.dm.off + (g.y0 + r) * W + g.x0 + cq + b] : (uint32_t)kOutside;
            if (c == kNoData || c == kOutside) a[b] = 0u;
            else wait_in |= (wv4[b] & kPMask) != 0u;
            if (in) O[r * W + cq + b] = a[b];
          }
        }
      }
    }
    WSTAMP(7);
    // ---- perimeter records
    const int64_t sb0 = g.tile * cap;
#pragma unroll
    for (int sI = 0; sI < NPS; ++sI) {
      const int j = tid + NT * sI;
      if (j >= cap) continue;
      const uint8_t ec = j < np ? pex(j) : (uint8_t)0xFF;
      if (ec != 0xFF) {
        int lr, lc;
        perim_cell(j, tw, th, lr, lc);
        ex_val[sb0 + j] = (uint64_t)((wd[widx(lr, lc)] & kAccMask) + 1u);
      }
      ex_code[sb0 + j] = ec;
    }
    for (uint32_t k = tid; k < nrq; k += NT) {
      const uint32_t e = rend[k];
      uint16_t link = 0xFFFF;
      if (e != 0xFFFFu) link = (uint16_t)perim_slot(T - (int)(e / S), (int)(e % S) - 4, tw, th);
      rl[sb0 + rq[k]] = link;
    }
    WSTAMP(8);
#ifdef D8_WALK_STAMPS
    if (lane == 0) {
      unsigned long long* acc = reinterpret_cast<unsigned long long*>(status + 800);
      for (int i = 0; i < 8; ++i) atomicAdd(acc + i, (unsigned long long)(wts_[i + 1] - wts_[i]));
      atomicAdd(status + 840, nbulk_);
      atomicAdd(status + 841, ntail_);
      atomicAdd(status + 842, 1u);
    }
#endif
    if (tid > 0 && tid < 8) cnt[tid] = 0u;
    lds_barrier();  // LDS reused by the next tile
    cur = nxt;
    g = gn;
    tc = tn;
  }
  if (badd) set_status(status, kStBadDir);
  if (cyc) set_status(status, kStCycle);
  if (wait_in) set_status(status, kStCycle);
}

__global__ void k_zero_words(uint32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

hipError_t launch_walk_count(const Plan& p, const uint8_t* dirs, uint32_t* out, int wpt, hipStream_t s) {
  const int64_t nt = p.span ? p.span : p.ntiles;
  const int64_t f = p.span ? p.first : (int64_t)0;
  uint32_t* ctr = p.hdr + 16;  // eight per-XCD tile counters
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, ctr, 8);
  // as many workgroups as the GPU keeps resident (LDS: seven per CU), or
  // one per tile
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
#ifndef D8_WALK_RESIDENT
#define D8_WALK_RESIDENT 7
#endif
  const int64_t grid = D8_WALK_RESIDENT > 0 ? std::min<int64_t>(nt, (int64_t)ncu * D8_WALK_RESIDENT) : nt;
  if (wpt == 4)
    hipLaunchKernelGGL(k_walk_count<4>, dim3((unsigned)grid), dim3(256), 0, s, dirs, p.tab, nt, p.cap, p.ex_code,
                       p.rl, p.ex_val, out, p.hdr, f, ctr);
  else if (wpt == 2)
    hipLaunchKernelGGL(k_walk_count<2>, dim3((unsigned)grid), dim3(128), 0, s, dirs, p.tab, nt, p.cap, p.ex_code,
                       p.rl, p.ex_val, out, p.hdr, f, ctr);
  else
    hipLaunchKernelGGL(k_walk_count<1>, dim3((unsigned)grid), dim3(64), 0, s, dirs, p.tab, nt, p.cap, p.ex_code,
                       p.rl, p.ex_val, out, p.hdr, f, ctr);
  return hipGetLastError();
}

}  // namespace d8
