// Host-side plan of one accumulation call and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stddef.h>
#include <stdint.h>

#include "d8_dev.hpp"

namespace d8 {

// Workspace layout (all offsets 256-byte aligned):
//   header   4096 B: [0] status word, [1] final-buffer index of the forward
//            resolve, [2] of the backward resolve, [3] super-block exit
//            nodes, [4] nodes in plist, [64..127] round flags
//   demtab   DemInfo x ndem                (batched calls only)
//   ex_code  uint8  x nslots   direction code of an exit slot, 0xFF otherwise
//   rl       uint16 x nslots   receiver slot -> exit slot of its in-tile path
//   ex_val   8 B    x nslots   exit partial value (forward) / receiver path
//                              sum (backward)
//   buf[3]   8 B    x nnode, nnode, nslots   resolve values (forward: [0]
//                              values of the super-block exits by dense node
//                              id, [1] and [2] their pending increments; [2]
//                              then the inflow of every receiver slot)
//   anc[2]   int32  x nnode, nslots   resolve ancestor pointers (forward:
//                              anc[0] the nodes' ancestors by node id, anc[1]
//                              every tile exit's super-block root node id)
//   list     int32  x nnode    forward: second ancestor buffer of the nodes;
//                              backward: exit list of even rounds
//   plist    int32  x nnode    forward: the nodes taking part in the doubling
//                              stage of the global resolve; backward: exit
//                              list of odd rounds (the backward layout pads
//                              both lists by list_pad() entries)
// nnode: the forward's level-2 nodes, at most one per super-block perimeter
// cell (nsb * 4 * kSuper); the backward indexes these arrays by exit slot
// (nnode = nslots).
//   lcnt     uint32 x 2 kListGrid   backward: per workgroup, the length of its
//                              segment of the two exit lists
//   blo      float  x ncells   backward: per cell, the low part of its fp64
//                              in-tile path sum (the high part is held in the
//                              output between the two tile passes)
//   broot    uint16 x ncells   backward: per cell, the perimeter index of the
//                              exit its in-tile path leaves by (0xFFFF: none);
//                              both by packed cell index (absent when ncells
//                              = 0, the forward calls' layout)
// A slot is one perimeter cell of one tile: slot id = tile * cap + perimeter
// index (see perim_slot).
struct Plan {
  int ts = 0;        // tile side
  int cap = 0;       // perimeter slots per tile (4*ts - 4)
  int64_t ntiles = 0;
  int64_t nslots = 0;
  int rounds = 0;    // resolve rounds (ceil(log2(nslots+1)) + 1)
  int bw = 0, bh = 0;  // workgroup block of the tile passes (whole tiles)
  int cpt = 16;        // cells per thread of the tile passes
  const float* dem = nullptr;  // fused call: codes computed from this DEM in the emit pass
  int wpt = 0;        // counts, 64 x 64 tiles: waves per tile of the walk pass (0: the doubling pass)
  // Streamed calls: when span > 0 the tile passes run only blocks (= tiles,
  // for 64 x 64 tiles and blocks) first .. first + span - 1.
  int64_t first = 0, span = 0;
  int64_t nblocks = 0;
  int64_t nsb = 0;     // super-blocks (kSuper x kSuper cells)
  int32_t* list = nullptr;  // second ancestor buffer of the super-block exit nodes
  int32_t* plist = nullptr;  // nodes of the doubling stage of the global resolve
  uint32_t* lcnt = nullptr;  // backward: segment lengths of the exit lists
  DemTable tab{};
  uint32_t* hdr = nullptr;
  DemInfo* demtab = nullptr;
  uint8_t* ex_code = nullptr;
  uint16_t* rl = nullptr;
  uint64_t* ex_val = nullptr;
  uint64_t* buf[3] = {nullptr, nullptr, nullptr};
  int32_t* anc[2] = {nullptr, nullptr};
  float* blo = nullptr;
  uint16_t* broot = nullptr;
  size_t bytes = 0;
};

constexpr size_t kHdrBytes = 4096;
// Backward resolve: list_grid() workgroups (one per 256 slots, at most
// kListGrid: enough threads in flight for its chains of dependent loads), each
// with a segment of the exit lists of list_segment() entries (a multiple of
// its 256 threads), so the lists need list_pad() entries beyond nslots.
constexpr int kListGrid = 16384;
inline int64_t list_grid(int64_t nslots) { return std::min<int64_t>((nslots + 255) / 256, kListGrid); }
inline int64_t list_pad(int64_t nslots) { return list_grid(nslots) * 256; }
inline int64_t list_segment(int64_t nslots, int64_t grid) {
  const int64_t per = (nslots + grid * 256 - 1) / (grid * 256);
  return per * 256;
}
constexpr int kMaxRounds = 62;

// nsb: super-blocks (bounds the forward's level-2 nodes); ncells: packed
// cells the backward's per-cell arrays cover (0: the forward layout).
size_t plan_layout(Plan& p, int64_t ntiles, int ts, int ndem, int64_t nsb, int64_t ncells, void* base);

// Launchers (return hipError_t of the last launch).
// Flow directions over 64x64-cell blocks (tab built with tile side 64).
constexpr int kFlowdirsBlock = 64;
hipError_t launch_flowdirs(const float* dem, uint8_t* dirs, const DemTable& tab, int64_t nblocks, hipStream_t s,
                           bool steepest = false);
hipError_t launch_build_demtab(const void* desc_dev, int32_t n, int ts, int bw, int bh, DemInfo* out,
                               hipStream_t s);
// Workgroup shape of the tile passes for a tile side and `waves` (waves_ok).
void count_block_dims(int ts, int waves, int& bw, int& bh);
// Whether `waves` (0 = default) names a tile-pass launch shape for tile side
// ts; counts additionally accept the walk pass (tile 64, waves 1, 2, 4).
bool waves_ok(int ts, int waves, bool counts);
hipError_t launch_zero_header(uint32_t* hdr, hipStream_t s);

// Counts tile pass with unknown inflows by last-arriver walks (64 x 64 tiles).
hipError_t launch_walk_count(const Plan& p, const uint8_t* dirs, uint32_t* out, int wpt, hipStream_t s);
hipError_t launch_count_tiles(const Plan& p, const uint8_t* dirs, bool final_pass, uint32_t* out, hipStream_t s);
hipError_t launch_weighted_tiles(const Plan& p, const uint8_t* dirs, const float* w, bool final_pass,
                                 float* out, float* out_lo, hipStream_t s);
hipError_t launch_backward_tiles(const Plan& p, const uint8_t* dirs, const float* g, bool final_pass,
                                 float* out, hipStream_t s);
hipError_t launch_forward_resolve(const Plan& p, bool weighted, hipStream_t s);
hipError_t launch_backward_resolve(const Plan& p, hipStream_t s);

// Epsilon fill over 64x64 tiles.  Workspace: cnt (words 0-2: the queue
// lengths of three rotating rounds; 3: the number of rounds that had work;
// 4-6: the rounds' tile-grab counters), qround
// (per tile: the last round it was queued for) and two tile queues.
constexpr int kFillTile = 64;
struct FillArgs {
  const float* z = nullptr;
  float* F = nullptr;
  int64_t H = 0, W = 0, TX = 0, TY = 0;
  float eps = 0.0f;
  uint32_t* cnt = nullptr;
  uint32_t* qround = nullptr;
  uint32_t* queue[2] = {nullptr, nullptr};
};
hipError_t launch_fill_reset(const FillArgs& a, hipStream_t s);
hipError_t launch_fill_round(const FillArgs& a, uint32_t round, hipStream_t s);

}  // namespace d8
