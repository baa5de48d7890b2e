// Device-side helpers shared by the gfx950 kernels of the D8 library.
//
// Direction codes: 0 E, 1 NE, 2 N, 3 NW, 4 W, 5 SW, 6 S, 7 SE, 8 outlet,
// 255 NoData (row 0 = north).  Code i drains to offset (ddr(i), ddc(i)); a
// neighbour at offset i drains into the centre cell iff its code is (i+4)&7.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d8 {

constexpr uint8_t kNone = 8;
constexpr uint8_t kNoData = 255;
constexpr uint8_t kOutside = 254;  // halo cell beyond the DEM edge (LDS only)

// Status word bits (workspace word 0).
constexpr uint32_t kStBadDir = 1u;
constexpr uint32_t kStCycle = 2u;

// Offsets from packed 2-bit tables (value + 1), branch-free; k in 0..7.
__device__ __forceinline__ int ddr_t(uint32_t k) { return (int)((0xA901u >> (2 * k)) & 3u) - 1; }
__device__ __forceinline__ int ddc_t(uint32_t k) { return (int)((0x901Au >> (2 * k)) & 3u) - 1; }

// Offsets as small lookup functions (no memory traffic): rows then cols.
__device__ __forceinline__ int ddr(int k) {
  // k: 0 E 0, 1 NE -1, 2 N -1, 3 NW -1, 4 W 0, 5 SW +1, 6 S +1, 7 SE +1
  return (k >= 1 && k <= 3) ? -1 : ((k >= 5) ? 1 : 0);
}
__device__ __forceinline__ int ddc(int k) {
  // k: 0 E +1, 1 NE +1, 2 N 0, 3 NW -1, 4 W -1, 5 SW -1, 6 S 0, 7 SE +1
  return (k == 0 || k == 1 || k == 7) ? 1 : ((k >= 3 && k <= 5) ? -1 : 0);
}

// ------------------------------------------------------------ tile geometry --
// Perimeter slots of a tw x th tile (tw, th >= 1): top row, bottom row, left
// column without corners, right column without corners.  These are the
// paper's "edge cells" of a partition (Sec. 3), generalised from strips to
// tiles.
__device__ __forceinline__ int perim_count(int tw, int th) {
  return th == 1 ? tw : (tw == 1 ? th : 2 * tw + 2 * (th - 2));
}
__device__ __forceinline__ bool on_perim(int r, int c, int tw, int th) {
  return r == 0 || c == 0 || r == th - 1 || c == tw - 1;
}
__device__ __forceinline__ int perim_slot(int r, int c, int tw, int th) {
  if (r == 0) return c;
  if (r == th - 1) return tw + c;
  if (c == 0) return 2 * tw + r - 1;
  return 2 * tw + (th - 2) + r - 1;  // c == tw - 1
}
__device__ __forceinline__ void perim_cell(int j, int tw, int th, int& r, int& c) {
  if (j < tw) { r = 0; c = j; return; }
  if (j < 2 * tw) { r = th - 1; c = j - tw; return; }
  if (j < 2 * tw + th - 2) { r = j - 2 * tw + 1; c = 0; return; }
  r = j - 2 * tw - (th - 2) + 1;
  c = tw - 1;
}

// One DEM of a (possibly single-element) batch, as the kernels see it.
struct DemInfo {
  int64_t off;      // element offset of cell (0,0) in the packed arrays
  int32_t H, W;     // shape
  int32_t TY, TX;   // tile grid
  int64_t tile0;    // first tile id of this DEM in the combined tile space
  int32_t BY, BX;   // grid of workgroup blocks (a block holds whole tiles)
  int64_t blk0;     // first block id of this DEM in the combined block space
  int32_t SBY, SBX; // grid of super-blocks (kSuper x kSuper cells of whole tiles)
  int64_t sb0;      // first super-block id of this DEM
};

// Side, in cells, of the super-blocks in which the tile-exit forest is
// resolved locally before the global resolve.
constexpr int kSuper = 256;

struct DemTable {
  const DemInfo* dev;  // device table (n > 1), sorted by tile0
  int32_t n;
  DemInfo one;         // used when n == 1
};

__device__ __forceinline__ DemInfo dem_of_block(const DemTable& t, int64_t blk) {
  if (t.n == 1) return t.one;
  int lo = 0, hi = t.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (t.dev[mid].blk0 <= blk) lo = mid; else hi = mid - 1;
  }
  return t.dev[lo];
}

__device__ __forceinline__ DemInfo dem_of_sb(const DemTable& t, int64_t sb) {
  if (t.n == 1) return t.one;
  int lo = 0, hi = t.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (t.dev[mid].sb0 <= sb) lo = mid; else hi = mid - 1;
  }
  return t.dev[lo];
}

__device__ __forceinline__ DemInfo dem_of_tile(const DemTable& t, int64_t tile) {
  if (t.n == 1) return t.one;
  int lo = 0, hi = t.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (t.dev[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return t.dev[lo];
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
  // tile index within its DEM: below 2^32 (a DEM has fewer than 2^32 cells),
  // so a 32-bit division
  const uint32_t lt = (uint32_t)(tile - g.dm.tile0);
  const uint32_t ty = lt / (uint32_t)g.dm.TX, tx = lt - ty * (uint32_t)g.dm.TX;
  g.y0 = (int64_t)ty * ts;
  g.x0 = (int64_t)tx * ts;
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

__device__ __forceinline__ void set_status(uint32_t* st, uint32_t bit) {
  __hip_atomic_fetch_or(st, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace d8
