// C ABI of the D8 library: argument checks, workspace layout, launch order.
// Every entry point only enqueues on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "d8.h"
#include "d8_internal.hpp"

namespace d8 {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t plan_layout(Plan& p, int64_t ntiles, int ts, int ndem, int64_t nsb, int64_t ncells, void* base) {
  p.ts = ts;
  p.cap = 4 * ts - 4;
  p.ntiles = ntiles;
  p.nslots = ntiles * p.cap;
  int r = 1;
  while (((int64_t)1 << (r - 1)) <= p.nslots && r < kMaxRounds) ++r;
  p.rounds = r;  // 2^(rounds-2) > nslots >= depth of the exit forest
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_hdr = take(kHdrBytes);
  const size_t o_tab = take(sizeof(DemInfo) * (size_t)std::max(ndem, 1));
  const size_t o_code = take((size_t)p.nslots);
  const size_t o_rl = take((size_t)p.nslots * 2);
  const size_t o_val = take((size_t)p.nslots * 8);
  // The forward's level-2 arrays (buf[0], buf[1], anc[0], list, plist) are
  // indexed by super-block exit node: at most one per super-block perimeter
  // cell.  The backward (ncells > 0) indexes them by exit slot, and pads the
  // two lists for its segmented exit lists.
  const int64_t nnode = ncells > 0 ? p.nslots : std::min<int64_t>(p.nslots, nsb * 4 * kSuper);
  const int64_t pad = ncells > 0 ? list_pad(p.nslots) : 0;
  size_t o_buf[3], o_anc[2];
  o_buf[0] = take((size_t)nnode * 8);
  o_buf[1] = take((size_t)nnode * 8);
  o_buf[2] = take((size_t)p.nslots * 8);  // also the inflow of every receiver slot
  o_anc[0] = take((size_t)nnode * 4);
  o_anc[1] = take((size_t)p.nslots * 4);  // every tile exit's super-block root
  const size_t o_list = take((size_t)(nnode + pad) * 4);
  const size_t o_plist = take((size_t)(nnode + pad) * 4);
  const size_t o_lcnt = ncells > 0 ? take((size_t)2 * kListGrid * 4) : 0;
  const size_t o_blo = ncells > 0 ? take((size_t)ncells * 4) : 0;
  const size_t o_broot = ncells > 0 ? take((size_t)ncells * 2) : 0;
  p.bytes = off;
  if (base) {
    char* b = static_cast<char*>(base);
    p.hdr = reinterpret_cast<uint32_t*>(b + o_hdr);
    p.demtab = reinterpret_cast<DemInfo*>(b + o_tab);
    p.ex_code = reinterpret_cast<uint8_t*>(b + o_code);
    p.rl = reinterpret_cast<uint16_t*>(b + o_rl);
    p.ex_val = reinterpret_cast<uint64_t*>(b + o_val);
    for (int i = 0; i < 3; ++i) p.buf[i] = reinterpret_cast<uint64_t*>(b + o_buf[i]);
    for (int i = 0; i < 2; ++i) p.anc[i] = reinterpret_cast<int32_t*>(b + o_anc[i]);
    p.list = reinterpret_cast<int32_t*>(b + o_list);
    p.plist = reinterpret_cast<int32_t*>(b + o_plist);
    p.lcnt = ncells > 0 ? reinterpret_cast<uint32_t*>(b + o_lcnt) : nullptr;
    p.blo = ncells > 0 ? reinterpret_cast<float*>(b + o_blo) : nullptr;
    p.broot = ncells > 0 ? reinterpret_cast<uint16_t*>(b + o_broot) : nullptr;
  }
  return p.bytes;
}

static int pick_tile(int tile) {
  if (tile == 0) return 64;
  if (tile == 32 || tile == 64 || tile == 128) return tile;
  return 0;
}

// At most 2^32 - 1 cells (uint32 counts and cell numbering) and at most
// 2^31 - 1 rows or columns (the kernels' DEM descriptor holds 32-bit sides).
static bool shape_ok(int64_t rows, int64_t cols) {
  return rows > 0 && cols > 0 && rows <= 0x7FFFFFFFll && cols <= 0x7FFFFFFFll &&
         (uint64_t)rows * (uint64_t)cols <= 0xFFFFFFFFull;
}

static DemInfo single_dem(int64_t rows, int64_t cols, int ts, int waves = 0) {
  DemInfo d;
  int bw, bh;
  count_block_dims(ts, waves, bw, bh);
  d.off = 0;
  d.H = (int32_t)rows;
  d.W = (int32_t)cols;
  d.TY = (int32_t)((rows + ts - 1) / ts);
  d.TX = (int32_t)((cols + ts - 1) / ts);
  d.tile0 = 0;
  d.BY = (int32_t)((rows + bh - 1) / bh);
  d.BX = (int32_t)((cols + bw - 1) / bw);
  d.blk0 = 0;
  d.SBY = (int32_t)((rows + kSuper - 1) / kSuper);
  d.SBX = (int32_t)((cols + kSuper - 1) / kSuper);
  d.sb0 = 0;
  return d;
}

// Launch shape of the tile passes for `waves` (waves_ok): cells per thread
// of the doubling passes on 64 x 64 tiles (64 / waves), or, for counts with
// waves 1, 2 or 4, the walk pass with that many waves per tile.
static void set_blocks(Plan& p, const d8_desc* hd, int32_t n, int64_t rows, int64_t cols, int waves,
                       bool counts = false) {
  count_block_dims(p.ts, waves, p.bw, p.bh);
  p.cpt = 16;
  if (p.ts == 64) p.cpt = waves >= 2 ? 64 / waves : 8;
  p.wpt = (counts && p.ts == 64 && (waves == 1 || waves == 2 || waves == 4)) ? waves : 0;
  p.nblocks = 0;
  p.nsb = 0;
  if (hd) {
    for (int32_t i = 0; i < n; ++i) {
      p.nblocks += ((int64_t)(hd[i].rows + p.bh - 1) / p.bh) * ((hd[i].cols + p.bw - 1) / p.bw);
      p.nsb += ((int64_t)(hd[i].rows + kSuper - 1) / kSuper) * ((hd[i].cols + kSuper - 1) / kSuper);
    }
  } else {
    p.nblocks = ((rows + p.bh - 1) / p.bh) * ((cols + p.bw - 1) / p.bw);
    p.nsb = ((rows + kSuper - 1) / kSuper) * ((cols + kSuper - 1) / kSuper);
  }
}

static d8_status hip_status(hipError_t e) { return e == hipSuccess ? D8_OK : D8_EHIP; }

// ------------------------------------------------------------ phase timing --
enum Phase {
  kPhFlowdirs = 0, kPhCountEmit, kPhCountResolve, kPhCountFinal, kPhWEmit, kPhWResolve, kPhWFinal,
  kPhBEmit, kPhBResolve, kPhBFinal
};
static const char* kPhaseNames[D8_NPHASES] = {
    "flowdirs", "count_tile_emit", "count_resolve", "count_tile_final", "weighted_tile_emit",
    "weighted_resolve", "weighted_tile_final", "backward_tile_emit", "backward_resolve", "backward_tile_final"};

struct PhaseRec {
  int phase;
  hipEvent_t a, b;
};
static bool g_timing = false;
static std::vector<PhaseRec> g_pending;
static std::vector<hipEvent_t> g_pool;
static double g_ms[D8_NPHASES];
static int g_calls[D8_NPHASES];

static hipEvent_t ev_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct PhaseScope {
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseScope(int phase, hipStream_t st) : ph(phase), s(st) {
    if (g_timing && (a = ev_get()) != nullptr && hipEventRecord(a, s) != hipSuccess) {
      g_pool.push_back(a);
      a = nullptr;
    }
  }
  ~PhaseScope() {
    if (!a) return;
    hipEvent_t b = ev_get();
    if (b && hipEventRecord(b, s) == hipSuccess) {
      g_pending.push_back({ph, a, b});
    } else {
      g_pool.push_back(a);
      if (b) g_pool.push_back(b);
    }
  }
};

static void drain_pending() {
  for (auto& r : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_ms[r.phase] += ms;
      g_calls[r.phase] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_pending.clear();
}

}  // namespace d8

using namespace d8;

extern "C" {

const char* d8_version(void) { return "d8-gfx950 0.1"; }

const char* d8_strerror(d8_status s) {
  switch (s) {
    case D8_OK: return "ok";
    case D8_EINVAL: return "invalid argument";
    case D8_ENOMEM: return "workspace too small";
    case D8_EHIP: return "HIP runtime error";
    case D8_EBADDIR: return "invalid direction field (bad code, or a target off the grid or into NoData)";
    case D8_ECYCLE: return "direction field contains a cycle";
    case D8_EUNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

static d8_status flowdirs_rule(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, void* stream,
                               bool steepest) {
  if (!dem || !dirs || !shape_ok(rows, cols)) return D8_EINVAL;
  DemTable tab{};
  tab.n = 1;
  tab.one = single_dem(rows, cols, kFlowdirsBlock);
  const int64_t nb = (int64_t)tab.one.TY * tab.one.TX;
  PhaseScope ps(kPhFlowdirs, (hipStream_t)stream);
  return hip_status(launch_flowdirs(dem, dirs, tab, nb, (hipStream_t)stream, steepest));
}

d8_status d8_flowdirs(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, void* stream) {
  return flowdirs_rule(dem, rows, cols, dirs, stream, false);
}

d8_status d8_flowdirs_steepest(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, void* stream) {
  return flowdirs_rule(dem, rows, cols, dirs, stream, true);
}

static int64_t super_blocks(int64_t rows, int64_t cols) {
  return ((rows + kSuper - 1) / kSuper) * ((cols + kSuper - 1) / kSuper);
}

size_t d8_workspace_bytes(int64_t rows, int64_t cols, int tile) {
  const int ts = pick_tile(tile);
  if (!ts || !shape_ok(rows, cols)) return 0;
  Plan p;
  const int64_t nt = ((rows + ts - 1) / ts) * ((cols + ts - 1) / ts);
  return plan_layout(p, nt, ts, 1, super_blocks(rows, cols), 0, nullptr);
}

size_t d8_backward_workspace_bytes(int64_t rows, int64_t cols, int tile) {
  const int ts = pick_tile(tile);
  if (!ts || !shape_ok(rows, cols)) return 0;
  Plan p;
  const int64_t nt = ((rows + ts - 1) / ts) * ((cols + ts - 1) / ts);
  return plan_layout(p, nt, ts, 1, super_blocks(rows, cols), rows * cols, nullptr);
}

// backward: the workspace also holds the per-cell exit array.
static d8_status prep_single(Plan& p, int64_t rows, int64_t cols, void* ws, size_t ws_bytes, int tile,
                             bool backward = false) {
  const int ts = pick_tile(tile);
  if (!ts || !shape_ok(rows, cols) || !ws) return D8_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return D8_EINVAL;
  const int64_t nt = ((rows + ts - 1) / ts) * ((cols + ts - 1) / ts);
  const int64_t nc = backward ? rows * cols : 0;
  if (plan_layout(p, nt, ts, 1, super_blocks(rows, cols), nc, nullptr) > ws_bytes) return D8_ENOMEM;
  plan_layout(p, nt, ts, 1, super_blocks(rows, cols), nc, ws);
  set_blocks(p, nullptr, 1, rows, cols, 0);
  p.tab.n = 1;
  p.tab.dev = nullptr;
  p.tab.one = single_dem(rows, cols, ts);
  return D8_OK;
}

static d8_status run_forward(const Plan& p, const uint8_t* dirs, const float* w, d8_dtype out_dtype, void* out,
                             float* out_lo, hipStream_t s) {
  hipError_t e = launch_zero_header(p.hdr, s);
  if (e != hipSuccess) return D8_EHIP;
  if (out_dtype == D8_U32) {
    {
      PhaseScope ps(kPhCountEmit, s);
      if ((e = launch_count_tiles(p, dirs, false, static_cast<uint32_t*>(out), s)) != hipSuccess) return D8_EHIP;
    }
    {
      PhaseScope ps(kPhCountResolve, s);
      if ((e = launch_forward_resolve(p, false, s)) != hipSuccess) return D8_EHIP;
    }
    {
      PhaseScope ps(kPhCountFinal, s);
      if ((e = launch_count_tiles(p, dirs, true, static_cast<uint32_t*>(out), s)) != hipSuccess) return D8_EHIP;
    }
  } else {
    if (p.ts > 64) return D8_EUNSUPPORTED;
    {
      PhaseScope ps(kPhWEmit, s);
      if ((e = launch_weighted_tiles(p, dirs, w, false, static_cast<float*>(out), out_lo, s)) != hipSuccess)
        return D8_EHIP;
    }
    {
      PhaseScope ps(kPhWResolve, s);
      if ((e = launch_forward_resolve(p, true, s)) != hipSuccess) return D8_EHIP;
    }
    {
      PhaseScope ps(kPhWFinal, s);
      if ((e = launch_weighted_tiles(p, dirs, w, true, static_cast<float*>(out), out_lo, s)) != hipSuccess)
        return D8_EHIP;
    }
  }
  return D8_OK;
}

static d8_status run_backward(const Plan& p, const uint8_t* dirs, const float* g, float* gw, hipStream_t s) {
  if (p.ts > 64) return D8_EUNSUPPORTED;
  if (!p.broot || !p.blo || !p.lcnt) return D8_EINVAL;
  hipError_t e = launch_zero_header(p.hdr, s);
  if (e != hipSuccess) return D8_EHIP;
  {
    PhaseScope ps(kPhBEmit, s);
    if ((e = launch_backward_tiles(p, dirs, g, false, gw, s)) != hipSuccess) return D8_EHIP;
  }
  {
    PhaseScope ps(kPhBResolve, s);
    if ((e = launch_backward_resolve(p, s)) != hipSuccess) return D8_EHIP;
  }
  {
    PhaseScope ps(kPhBFinal, s);
    if ((e = launch_backward_tiles(p, dirs, g, true, gw, s)) != hipSuccess) return D8_EHIP;
  }
  return D8_OK;
}

d8_status d8_accum(const uint8_t* dirs, int64_t rows, int64_t cols, const float* weights, d8_dtype out_dtype,
                   void* out, float* out_lo, void* ws, size_t ws_bytes, int tile, void* stream) {
  if (!dirs || !out) return D8_EINVAL;
  if (out_dtype != D8_U32 && out_dtype != D8_F32) return D8_EINVAL;
  if (out_dtype == D8_U32 && (weights || out_lo)) return D8_EINVAL;
  Plan p;
  d8_status st = prep_single(p, rows, cols, ws, ws_bytes, tile);
  if (st != D8_OK) return st;
  if (out_dtype == D8_F32 && p.ts > 64) return D8_EUNSUPPORTED;
  return run_forward(p, dirs, weights, out_dtype, out, out_lo, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------- no-alloc --
namespace d8 {
// The workspace of d8_accum_noalloc: a static device array, one copy per GPU
// that loads the library.  Host code must use its device address (from
// hipGetSymbolAddress on the current device), never the symbol itself.
static __device__ __align__(256) uint8_t scratch[D8_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::atomic<void*> g_scratch[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per
// device), or nullptr if the lookup fails.
static void* scratch_here() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  void* p = g_scratch[dev].load(std::memory_order_acquire);
  if (p) return p;
  void* q = nullptr;
  if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return nullptr;
  g_scratch[dev].store(q, std::memory_order_release);
  return q;
}

__global__ void k_copy_status(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}
}  // namespace d8

extern "C" {

d8_status d8_accum_noalloc(const uint8_t* dirs, int64_t rows, int64_t cols, const float* weights,
                           d8_dtype out_dtype, void* out, float* out_lo, int tile, uint32_t* status,
                           void* stream) {
  if (!dirs || !out) return D8_EINVAL;
  if (out_dtype != D8_U32 && out_dtype != D8_F32) return D8_EINVAL;
  if (out_dtype == D8_U32 && (weights || out_lo)) return D8_EINVAL;
  const size_t need = d8_workspace_bytes(rows, cols, tile);
  if (!need) return D8_EINVAL;
  if (need > (size_t)D8_NOALLOC_SCRATCH_BYTES) return D8_ENOMEM;
  void* ws = scratch_here();
  if (!ws) return D8_EHIP;
  Plan p;
  d8_status st = prep_single(p, rows, cols, ws, (size_t)D8_NOALLOC_SCRATCH_BYTES, tile);
  if (st != D8_OK) return st;
  if (out_dtype == D8_F32 && p.ts > 64) return D8_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  st = run_forward(p, dirs, weights, out_dtype, out, out_lo, s);
  if (st != D8_OK || !status) return st;
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, p.hdr, status);
  return hip_status(hipGetLastError());
}

d8_status d8_accum_dem(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, uint32_t* out, void* ws,
                       size_t ws_bytes, int tile, void* stream) {
  if (!dem || !dirs || !out) return D8_EINVAL;
  Plan p;
  d8_status st = prep_single(p, rows, cols, ws, ws_bytes, tile);
  if (st != D8_OK) return st;
  p.dem = dem;  // the emit pass computes (and writes) the codes
  return run_forward(p, dirs, nullptr, D8_U32, out, nullptr, (hipStream_t)stream);
}

d8_status d8_accum_backward(const uint8_t* dirs, int64_t rows, int64_t cols, const float* grad_out,
                            float* grad_weights, void* ws, size_t ws_bytes, int tile, void* stream) {
  if (!dirs || !grad_out || !grad_weights) return D8_EINVAL;
  Plan p;
  d8_status st = prep_single(p, rows, cols, ws, ws_bytes, tile, true);
  if (st != D8_OK) return st;
  if (p.ts > 64) return D8_EUNSUPPORTED;
  return run_backward(p, dirs, grad_out, grad_weights, (hipStream_t)stream);
}

// ----------------------------------------------------------------- streamed --
// Host-resident direction field and counts: row strips of `strip_rows` rows
// pass through the device twice, once for the tile pass with unknown inflows
// and once for the finalising pass; the perimeter records and the resolve
// stay on the device for the whole DEM.  Two strip slots and two copy
// streams (host to device, device to host) let the copies of neighbouring
// strips run under the kernels of the current one and in both directions at
// once; events order each slot's reuse.

static size_t streamed_plan_bytes(int64_t rows, int64_t cols) { return d8_workspace_bytes(rows, cols, 64); }
static size_t strip_dirs_bytes(int64_t sr, int64_t cols) { return align256((size_t)(sr + 2) * (size_t)cols); }
static size_t strip_out_bytes(int64_t sr, int64_t cols) { return align256((size_t)sr * (size_t)cols * 4); }

size_t d8_accum_streamed_workspace_bytes(int64_t rows, int64_t cols, int64_t strip_rows) {
  if (!shape_ok(rows, cols) || strip_rows <= 0 || strip_rows % 64) return 0;
  const int64_t sr = std::min<int64_t>(strip_rows, (rows + 63) / 64 * 64);
  return streamed_plan_bytes(rows, cols) + 2 * (strip_dirs_bytes(sr, cols) + strip_out_bytes(sr, cols));
}

namespace {
// Streams and events of one streamed call, released on every return path.
struct StreamSet {
  hipStream_t in = nullptr, out = nullptr;
  hipEvent_t start = nullptr, pass1 = nullptr, last = nullptr;
  hipEvent_t loaded[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr}, stored[2] = {nullptr, nullptr};
  bool ok = true;
  StreamSet() {
    ok = hipStreamCreateWithFlags(&in, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&out, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* e : {&start, &pass1, &last, &loaded[0], &loaded[1], &done[0], &done[1], &stored[0], &stored[1]})
      ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  }
  ~StreamSet() {
    for (hipEvent_t e : {start, pass1, last, loaded[0], loaded[1], done[0], done[1], stored[0], stored[1]})
      if (e) (void)hipEventDestroy(e);
    if (in) (void)hipStreamDestroy(in);
    if (out) (void)hipStreamDestroy(out);
  }
};
}  // namespace

d8_status d8_accum_streamed(const uint8_t* dirs_host, int64_t rows, int64_t cols, uint32_t* out_host,
                            int64_t strip_rows, void* ws, size_t ws_bytes, void* stream) {
  if (!dirs_host || !out_host) return D8_EINVAL;
  const size_t need = d8_accum_streamed_workspace_bytes(rows, cols, strip_rows);
  if (!need || !ws) return D8_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return D8_EINVAL;
  if (ws_bytes < need) return D8_ENOMEM;
  const size_t pb = streamed_plan_bytes(rows, cols);
  Plan p;
  d8_status st = prep_single(p, rows, cols, ws, pb, 64);
  if (st != D8_OK) return st;
  if (p.bw != 64 || p.bh != 64) return D8_EUNSUPPORTED;  // blocks must be the tiles
  const int64_t sr = std::min<int64_t>(strip_rows, (rows + 63) / 64 * 64);
  uint8_t* dbuf[2];
  uint32_t* obuf[2];
  {
    uint8_t* b = static_cast<uint8_t*>(ws) + pb;
    for (int i = 0; i < 2; ++i) {
      dbuf[i] = b;
      b += strip_dirs_bytes(sr, cols);
      obuf[i] = reinterpret_cast<uint32_t*>(b);
      b += strip_out_bytes(sr, cols);
    }
  }
  const int64_t tx = (cols + 63) / 64;
  hipStream_t s = (hipStream_t)stream;
  StreamSet ss;
  if (!ss.ok) return D8_EHIP;
  // the workspace may still be in use by earlier work on `stream`
  if (hipEventRecord(ss.start, s) != hipSuccess || hipStreamWaitEvent(ss.in, ss.start, 0) != hipSuccess ||
      hipStreamWaitEvent(ss.out, ss.start, 0) != hipSuccess || launch_zero_header(p.hdr, s) != hipSuccess)
    return D8_EHIP;
  const auto fail = [&]() {
    (void)hipStreamSynchronize(ss.in);
    (void)hipStreamSynchronize(ss.out);
    (void)hipStreamSynchronize(s);
    return D8_EHIP;
  };
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      p.first = p.span = 0;
      if (launch_forward_resolve(p, false, s) != hipSuccess) return fail();
      // the finalising pass reads back the tile-local counts of the first
      if (hipEventRecord(ss.pass1, ss.out) != hipSuccess || hipStreamWaitEvent(ss.in, ss.pass1, 0) != hipSuccess)
        return fail();
    }
    int64_t strip = 0;
    for (int64_t s0 = 0; s0 < rows; s0 += sr, ++strip) {
      const int b = (int)(strip & 1);
      const int64_t s1 = std::min(rows, s0 + sr);
      const int64_t r0 = std::max<int64_t>(s0 - 1, 0), r1 = std::min(s1, rows - 1);  // rows with the halo
      // slot b is free once the strip two back has been copied out
      if (hipStreamWaitEvent(ss.in, ss.stored[b], 0) != hipSuccess ||
          hipMemcpyAsync(dbuf[b], dirs_host + r0 * cols, (size_t)(r1 - r0 + 1) * (size_t)cols,
                         hipMemcpyHostToDevice, ss.in) != hipSuccess)
        return fail();
      if (pass == 1 && hipMemcpyAsync(obuf[b], out_host + s0 * cols, (size_t)(s1 - s0) * (size_t)cols * 4,
                                      hipMemcpyHostToDevice, ss.in) != hipSuccess)
        return fail();
      if (hipEventRecord(ss.loaded[b], ss.in) != hipSuccess || hipStreamWaitEvent(s, ss.loaded[b], 0) != hipSuccess)
        return fail();
      // the strip's tile rows; buffers addressed by global cell index
      p.first = (s0 / 64) * tx;
      p.span = ((s1 - s0 + 63) / 64) * tx;
      if (launch_count_tiles(p, dbuf[b] - r0 * cols, pass == 1, obuf[b] - s0 * cols, s) != hipSuccess ||
          hipEventRecord(ss.done[b], s) != hipSuccess || hipStreamWaitEvent(ss.out, ss.done[b], 0) != hipSuccess ||
          hipMemcpyAsync(out_host + s0 * cols, obuf[b], (size_t)(s1 - s0) * (size_t)cols * 4, hipMemcpyDeviceToHost,
                         ss.out) != hipSuccess ||
          hipEventRecord(ss.stored[b], ss.out) != hipSuccess)
        return fail();
    }
  }
  if (hipEventRecord(ss.last, ss.out) != hipSuccess || hipStreamWaitEvent(s, ss.last, 0) != hipSuccess)
    return fail();
  const bool good = hipStreamSynchronize(ss.in) == hipSuccess && hipStreamSynchronize(ss.out) == hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess;
  return good ? D8_OK : D8_EHIP;
}

// ------------------------------------------------------------- conditioning --

static int64_t fill_tiles(int64_t rows, int64_t cols) {
  return ((rows + kFillTile - 1) / kFillTile) * ((cols + kFillTile - 1) / kFillTile);
}
size_t d8_fill_workspace_bytes(int64_t rows, int64_t cols) {
  if (!shape_ok(rows, cols)) return 0;
  return 256 + 3 * align256((size_t)fill_tiles(rows, cols) * sizeof(uint32_t));
}

d8_status d8_fill_eps(const float* dem, int64_t rows, int64_t cols, float eps, float* out, void* ws,
                      size_t ws_bytes, int64_t* rounds, void* stream) {
  if (!dem || !out || !ws || !shape_ok(rows, cols)) return D8_EINVAL;
  if (!(eps >= 1.17549435e-38f) || !std::isfinite(eps)) return D8_EINVAL;  // positive normal
  const size_t nb = (size_t)rows * (size_t)cols * sizeof(float);
  const char* zb = reinterpret_cast<const char*>(dem);
  const char* ob = reinterpret_cast<const char*>(out);
  if (ob < zb + nb && zb < ob + nb) return D8_EINVAL;  // out overlaps dem
  if (reinterpret_cast<uintptr_t>(ws) & 255) return D8_EINVAL;
  if (ws_bytes < d8_fill_workspace_bytes(rows, cols)) return D8_ENOMEM;
  const int64_t nt = fill_tiles(rows, cols);
  const size_t qb = align256((size_t)nt * sizeof(uint32_t));
  char* base = static_cast<char*>(ws);
  FillArgs a;
  a.z = dem;
  a.F = out;
  a.H = rows;
  a.W = cols;
  a.TY = (rows + kFillTile - 1) / kFillTile;
  a.TX = (cols + kFillTile - 1) / kFillTile;
  a.eps = eps;
  a.cnt = reinterpret_cast<uint32_t*>(base);
  a.qround = reinterpret_cast<uint32_t*>(base + 256);
  a.queue[0] = reinterpret_cast<uint32_t*>(base + 256 + qb);
  a.queue[1] = reinterpret_cast<uint32_t*>(base + 256 + 2 * qb);
  hipStream_t s = (hipStream_t)stream;
  if (launch_fill_reset(a, s) != hipSuccess) return D8_EHIP;
  // Round r drains queue r and fills queue r+1; the host looks at the length
  // of the next queue now and then (round 0 queues every tile once more).
  const uint32_t kMaxFillRounds = 1u << 24;
  for (uint32_t r = 0;; ++r) {
    if (launch_fill_round(a, r, s) != hipSuccess) return D8_EHIP;
    // look after rounds 1, 2, 4, 8 and then every 8th (a look idles the GPU
    // for a host round trip; a round past the end costs one empty launch)
    if (r == 0 || !(r <= 8 ? (r & (r - 1)) == 0 : r % 8 == 0)) continue;
    uint32_t next = 0;
    if (hipMemcpyAsync(&next, a.cnt + (r + 1) % 3, sizeof(next), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return D8_EHIP;
    if (next == 0) break;
    if (r >= kMaxFillRounds) return D8_ECYCLE;
  }
  if (rounds) {
    uint32_t used = 0;
    if (hipMemcpyAsync(&used, a.cnt + 3, sizeof(used), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return D8_EHIP;
    *rounds = used;
  }
  return D8_OK;
}

// ------------------------------------------------------------------ batched --

static bool batch_tiles(const d8_desc* hd, int32_t n, int ts, int64_t& ntiles) {
  ntiles = 0;
  if (!hd || n <= 0) return false;
  for (int32_t i = 0; i < n; ++i) {
    if (hd[i].rows <= 0 || hd[i].cols <= 0 || hd[i].offset < 0) return false;
    if ((int64_t)hd[i].rows * hd[i].cols > 0x7FFFFFFFll) return false;
    ntiles += ((int64_t)(hd[i].rows + ts - 1) / ts) * ((hd[i].cols + ts - 1) / ts);
  }
  return true;
}

// Extent of the packed cells: the largest offset + rows * cols.
static int64_t batch_span(const d8_desc* hd, int32_t n) {
  int64_t e = 0;
  for (int32_t i = 0; i < n; ++i) e = std::max<int64_t>(e, hd[i].offset + (int64_t)hd[i].rows * hd[i].cols);
  return e;
}

static int64_t batch_super_blocks(const d8_desc* hd, int32_t n) {
  int64_t b = 0;
  for (int32_t i = 0; i < n; ++i) b += super_blocks(hd[i].rows, hd[i].cols);
  return b;
}

size_t d8_batched_workspace_bytes(const d8_desc* host_desc, int32_t n, int tile) {
  const int ts = pick_tile(tile);
  int64_t nt;
  if (!ts || !batch_tiles(host_desc, n, ts, nt)) return 0;
  int64_t ntf;
  batch_tiles(host_desc, n, kFlowdirsBlock, ntf);
  Plan p;
  size_t b = plan_layout(p, nt, ts, n, batch_super_blocks(host_desc, n), 0, nullptr);
  return std::max(b, align256(kHdrBytes) + align256(sizeof(DemInfo) * (size_t)n));
}

size_t d8_batched_backward_workspace_bytes(const d8_desc* host_desc, int32_t n, int tile) {
  const int ts = pick_tile(tile);
  int64_t nt;
  if (!ts || !batch_tiles(host_desc, n, ts, nt)) return 0;
  Plan p;
  return plan_layout(p, nt, ts, n, batch_super_blocks(host_desc, n), batch_span(host_desc, n), nullptr);
}

static d8_status prep_batched(Plan& p, const d8_desc* hd, const d8_desc* dd, int32_t n, void* ws, size_t ws_bytes,
                              int ts, hipStream_t s, int waves = 0, bool counts = false, bool backward = false) {
  int64_t nt;
  if (!ts || !dd || !ws || !batch_tiles(hd, n, ts, nt)) return D8_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return D8_EINVAL;
  const int64_t nc = backward ? batch_span(hd, n) : 0;
  const int64_t nsb = batch_super_blocks(hd, n);
  if (plan_layout(p, nt, ts, n, nsb, nc, nullptr) > ws_bytes) return D8_ENOMEM;
  plan_layout(p, nt, ts, n, nsb, nc, ws);
  set_blocks(p, hd, n, 0, 0, waves, counts);
  if (n == 1) {
    p.tab.n = 1;
    p.tab.dev = nullptr;
    DemInfo d = single_dem(hd[0].rows, hd[0].cols, ts, waves);
    d.off = hd[0].offset;
    p.tab.one = d;
    return D8_OK;
  }
  p.tab.n = n;
  p.tab.dev = p.demtab;
  return hip_status(launch_build_demtab(dd, n, ts, p.bw, p.bh, p.demtab, s));
}

d8_status d8_flowdirs_batched(const float* dem_packed, const d8_desc* host_desc, const d8_desc* dev_desc, int32_t n,
                              uint8_t* dirs_packed, void* ws, size_t ws_bytes, void* stream) {
  if (!dem_packed || !dirs_packed) return D8_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Plan p;
  d8_status st = prep_batched(p, host_desc, dev_desc, n, ws, ws_bytes, kFlowdirsBlock, s);
  if (st == D8_ENOMEM) {
    // flowdirs needs only the header and the DEM table
    if (ws_bytes < align256(kHdrBytes) + align256(sizeof(DemInfo) * (size_t)n)) return D8_ENOMEM;
    int64_t nt;
    batch_tiles(host_desc, n, kFlowdirsBlock, nt);
    p = Plan();
    p.hdr = static_cast<uint32_t*>(ws);
    p.demtab = reinterpret_cast<DemInfo*>(static_cast<char*>(ws) + align256(kHdrBytes));
    p.ntiles = nt;
    if (n == 1) {
      p.tab.n = 1;
      p.tab.one = single_dem(host_desc[0].rows, host_desc[0].cols, kFlowdirsBlock);
      p.tab.one.off = host_desc[0].offset;
    } else {
      p.tab.n = n;
      p.tab.dev = p.demtab;
      if (launch_build_demtab(dev_desc, n, kFlowdirsBlock, kFlowdirsBlock, kFlowdirsBlock, p.demtab, s) != hipSuccess)
        return D8_EHIP;
    }
  } else if (st != D8_OK) {
    return st;
  }
  return hip_status(launch_flowdirs(dem_packed, dirs_packed, p.tab, p.ntiles, s));
}

d8_status d8_accum_batched(const uint8_t* dirs_packed, const d8_desc* host_desc, const d8_desc* dev_desc, int32_t n,
                           const float* w_packed, d8_dtype out_dtype, void* out_packed, float* out_lo_packed,
                           void* ws, size_t ws_bytes, int tile, int waves, void* stream) {
  if (!dirs_packed || !out_packed) return D8_EINVAL;
  if (out_dtype != D8_U32 && out_dtype != D8_F32) return D8_EINVAL;
  if (out_dtype == D8_U32 && (w_packed || out_lo_packed)) return D8_EINVAL;
  if (waves < 0 || waves > 16) return D8_EINVAL;
  const int ts = pick_tile(tile);
  if (!ts) return D8_EINVAL;
  if (out_dtype == D8_F32 && ts > 64) return D8_EUNSUPPORTED;
  if (!waves_ok(ts, waves, out_dtype == D8_U32)) return D8_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  Plan p;
  d8_status st = prep_batched(p, host_desc, dev_desc, n, ws, ws_bytes, ts, s, waves, out_dtype == D8_U32);
  if (st != D8_OK) return st;
  return run_forward(p, dirs_packed, w_packed, out_dtype, out_packed, out_lo_packed, s);
}

d8_status d8_accum_backward_batched(const uint8_t* dirs_packed, const d8_desc* host_desc, const d8_desc* dev_desc,
                                    int32_t n, const float* g_packed, float* gw_packed, void* ws, size_t ws_bytes,
                                    int tile, int waves, void* stream) {
  if (!dirs_packed || !g_packed || !gw_packed) return D8_EINVAL;
  if (waves < 0 || waves > 16) return D8_EINVAL;
  const int ts = pick_tile(tile);
  if (!ts) return D8_EINVAL;
  if (ts > 64 || !waves_ok(ts, waves, false)) return D8_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  Plan p;
  d8_status st = prep_batched(p, host_desc, dev_desc, n, ws, ws_bytes, ts, s, waves, false, true);
  if (st != D8_OK) return st;
  return run_backward(p, dirs_packed, g_packed, gw_packed, s);
}

d8_status d8_autotune_batched(const uint8_t* dirs_packed, const d8_desc* host_desc, const d8_desc* dev_desc,
                              int32_t n, const float* w_packed, float* out_scratch, float* g_scratch, void* ws,
                              size_t ws_bytes, int* best_tile, int* best_waves, float* best_ms, void* stream) {
  if (!best_tile || !best_waves) return D8_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return D8_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return D8_EHIP;
  }
  // every (tile, waves) launch shape of the fp64 tile passes: tile 32 with 1,
  // 2 or 4 tiles per workgroup, tile 64 with 2..16 waves per tile (fp64
  // tiles of 128 or 256 cells do not fit the 160 KiB of LDS of a CU)
  const int tiles[2] = {32, 64};
  const int waves_opts[5] = {1, 2, 4, 8, 16};
  float best = 1e30f;
  int bt = 0, bw = 0;
  d8_status last = D8_OK;
  for (int ti = 0; ti < 2; ++ti) {
    for (int wi = 0; wi < 5; ++wi) {
      const int t = tiles[ti], w = waves_opts[wi];
      if (!waves_ok(t, w, false)) continue;
      float ms_best = 1e30f;
      bool ok = true;
      for (int rep = 0; rep < 3 && ok; ++rep) {
        (void)hipEventRecord(e0, s);
        d8_status a = d8_accum_batched(dirs_packed, host_desc, dev_desc, n, w_packed, D8_F32, out_scratch, nullptr,
                                       ws, ws_bytes, t, w, stream);
        d8_status b = d8_accum_backward_batched(dirs_packed, host_desc, dev_desc, n, out_scratch, g_scratch, ws,
                                                ws_bytes, t, w, stream);
        (void)hipEventRecord(e1, s);
        if (a != D8_OK || b != D8_OK) {
          ok = false;
          last = a != D8_OK ? a : b;
          break;
        }
        if (hipEventSynchronize(e1) != hipSuccess) {
          ok = false;
          last = D8_EHIP;
          break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_best = std::min(ms_best, ms);
      }
      if (ok && ms_best < best) {
        best = ms_best;
        bt = t;
        bw = w;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!bt) return last == D8_OK ? D8_EUNSUPPORTED : last;
  *best_tile = bt;
  *best_waves = bw;
  if (best_ms) *best_ms = best;
  return D8_OK;
}

d8_status d8_phase_timing(int enable) {
  drain_pending();
  if (enable) {
    for (int i = 0; i < D8_NPHASES; ++i) {
      g_ms[i] = 0.0;
      g_calls[i] = 0;
    }
  }
  g_timing = enable != 0;
  return D8_OK;
}

d8_status d8_phase_report(int phase, const char** name, float* total_ms, int32_t* calls) {
  if (phase < 0 || phase >= D8_NPHASES) return D8_EINVAL;
  drain_pending();
  if (name) *name = kPhaseNames[phase];
  if (total_ms) *total_ms = (float)g_ms[phase];
  if (calls) *calls = g_calls[phase];
  return D8_OK;
}

d8_status d8_device_status(const void* ws, void* stream, int32_t* status_out) {
  if (!ws || !status_out) return D8_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return D8_EHIP;
  uint32_t w = 0;
  if (hipMemcpy(&w, ws, 4, hipMemcpyDeviceToHost) != hipSuccess) return D8_EHIP;
  *status_out = (w & kStBadDir) ? D8_EBADDIR : ((w & kStCycle) ? D8_ECYCLE : D8_OK);
  return D8_OK;
}

}  // extern "C"
