// Depression and flat conditioning on the GPU: the epsilon fill.
//
// Sec. 3 of the paper assumes the DEM was conditioned before the method runs
// (pits raised to the level they drain at, flats given small elevation
// changes) and names no algorithm.  The fill computed here is the epsilon
// fill of Planchon & Darboux (2002): seeds (valid cells on the DEM boundary or
// 8-adjacent to NaN) keep z, and every other valid cell gets the unique
// fixed point
//     F(c) = max(z(c), min over valid neighbours n of inc(F(n))),
//     inc(x) = fl32(x + eps), or the next float above x if that rounds to x.
// Min and max are taken in the total order of the float bit patterns, so the
// result is bit-exact whatever order the updates run in.
//
// The fixed point is reached from above (F = +inf off the seeds) by chaotic
// relaxation, which converges to the same unique point for any update order.
// Work is organised as 64x64 tiles in LDS, the same partition-with-unknowns
// idea as the accumulation: a tile visit relaxes the tile given the current
// values of its one-cell halo, writes back what changed and queues for the
// next round the neighbouring tiles a changed border cell can still lower,
// and the tile itself while it is still changing.  Rounds repeat until no
// tile is queued; then every tile is at its fixed point given its halo, and
// the halos hold the final values, so the whole DEM is at the fixed point.
//
// Inside a tile the four waves of the workgroup sweep concurrently in the four
// axis directions (rows down, rows up, columns right, columns left; one cell
// per lane per step), so values travel up to 64 cells along any monotone
// run per sweep.  Updates lower a cell's key with an LDS atomic min, which
// keeps every value an upper bound of the fixed point while the waves race.
// A cell already at z is final (values only fall and never below z): no
// candidate lowers it.
#include <algorithm>
#include <atomic>

#include "d8_internal.hpp"

// Optional per-visit statistics for measurement builds (no-op here):
// D8_FILL_STAT(round, sweep sets, start clock) at the end of a tile visit.
#ifndef D8_FILL_STAT
#define D8_FILL_STAT(round, sets, t0)
#endif

namespace d8 {
namespace {

constexpr int kFT = 64;            // tile side
constexpr int kFK = kFT + 3;       // row stride of the key array (halo ring + 1 pad: odd)
constexpr int kFZ = kFT + 1;       // row stride of the elevation array (odd)
constexpr int kFThreads = 256;     // four waves
constexpr uint32_t kKeyInf = 0xFF800000u;   // key of +inf (a valid cell not reached yet)
constexpr uint32_t kKeyNone = 0xFFFFFFFFu;  // no cell: outside the DEM or NaN (above every key)
// Extra sweep sets per tile visit.  With none, a visit runs one set and a
// tile whose set changed anything simply goes round again: its next visit
// also sees its neighbours' newer values, and no set is spent only to find
// that nothing changes (8192^2 raw surface: 6.8 -> 4.7 ms against sweeping
// each visit to its local fixed point).
constexpr int kFillSweepCap = 0;

__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fval(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
// inc(x) for x finite or +-inf; eps is a positive normal float.
__device__ __forceinline__ float inc_eps(float x, float eps) {
  const float y = x + eps;
  if (y > x) return y;
  if (x == __builtin_inff()) return x;
  const uint32_t u = __float_as_uint(x);
  return __uint_as_float(x > 0.0f ? u + 1u : u - 1u);  // next float above x (x != 0 here)
}

// Thread layout of the global loads and stores: wave w (of four) takes rows
// w, w + 4, ..., its lane the column, so each wave touches one contiguous row
// segment per step and the per-step address offset is uniform.
constexpr int kHR = (kFT + 2 + 3) / 4;  // steps over the kFT+2 rows of the halo tile
constexpr int kTR = kFT / 4;            // steps over the kFT rows of the tile

// The halo tile of src, rows y0-1 .. y0+kFT, columns x0-1 .. x0+kFT (NaN
// outside the DEM): v[p] is column lane-1 of halo row 4p+w, e[p] (lanes 0
// and 1) column kFT-1+lane.  Every load is issued before any is used.
__device__ __forceinline__ void load_halo_tile(const float* __restrict__ src, int64_t y0, int64_t x0, int64_t H,
                                               int64_t W, float (&v)[kHR], float (&e)[kHR]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t gx = x0 - 1 + lane, gx2 = x0 + kFT - 1 + lane;
  const bool cx = gx >= 0 && gx < W, cx2 = lane < 2 && gx2 < W;
  const float* p0 = src + (y0 - 1 + w) * W;
#pragma unroll
  for (int p = 0; p < kHR; ++p) {
    const int64_t gy = y0 - 1 + 4 * p + w;
    const bool cy = 4 * p + w < kFT + 2 && gy >= 0 && gy < H;
    const float* row = p0 + (int64_t)(4 * p) * W;
    v[p] = cy && cx ? row[gx] : __builtin_nanf("");
    e[p] = cy && cx2 ? row[gx2] : __builtin_nanf("");
  }
}

// Position in the key array of the i-th cell of the halo ring (top row, bottom
// row, left column, right column).
__device__ __forceinline__ int ring_index(int j) {
  int r, c;
  if (j < kFT + 2) { r = 0; c = j; }
  else if (j < 2 * (kFT + 2)) { r = kFT + 1; c = j - (kFT + 2); }
  else if (j < 3 * (kFT + 2) - 2) { r = j - 2 * (kFT + 2) + 1; c = 0; }
  else { r = j - 3 * (kFT + 2) + 3; c = kFT + 1; }
  return r * kFK + c;
}

__device__ __forceinline__ void fill_enqueue(const FillArgs& a, uint32_t t, uint32_t next_round) {
  if (atomicMax(&a.qround[t], next_round) < next_round) {
    const uint32_t slot = atomicAdd(&a.cnt[next_round % 3], 1u);
    a.queue[next_round & 1][slot] = t;
  }
}

// One set of sweeps of a tile, the part of wave DIR (0: rows top to bottom,
// 1: rows bottom to top, 2: columns left to right, 3: columns right to left).
// The wave walks its 64 lines one per step, lane x at position x of the line.
// It keeps three lines in registers: the previous one as this wave left it (a
// lane's neighbours there come from the adjacent lanes by DPP wave shifts,
// the edge lanes keeping their halo cell), the current one and the next one.
// Each step reads the line two ahead (three keys per lane, issued a step
// before they are needed) and the key of z.  Values read earlier may be
// higher than the current ones (other waves lower them meanwhile); every key
// is an upper bound of the fixed point at all times, and a set that changes
// nothing reads a constant array, so the result is the same.  Cells that are
// NaN or outside the DEM have z key kKeyNone, which no candidate beats, so
// the step needs no validity test.  Returns whether a cell was lowered.
template <int DIR>
__device__ __forceinline__ bool sweep_lines(uint32_t* K, const uint32_t* Zk, uint32_t* moved, int lane, float eps) {
  constexpr bool kRows = DIR < 2;
  constexpr int sg = (DIR == 0 || DIR == 2) ? 1 : -1;  // line step
  constexpr int L0 = sg > 0 ? 0 : kFT - 1;              // first line
  constexpr int ls = kRows ? kFK : 1, xs = kRows ? 1 : kFK;  // key index steps: line, position
  constexpr int zls = kRows ? kFZ : 1, zxs = kRows ? 1 : kFZ;
  // key of FLT_MAX: inc of it is +inf, as inc of +inf is, so candidates from
  // no or unreached neighbours need no test of their own
  constexpr uint32_t kKeyMax = 0xFF7FFFFFu;
  // key index of line L0, position lane (lines and positions -1 and kFT: halo)
  const int b0 = (L0 + 1) * ls + (lane + 1) * xs;
  uint32_t p1 = K[b0 - sg * ls], p0 = K[b0 - sg * ls - xs], p2 = K[b0 - sg * ls + xs];
  uint32_t c1 = K[b0], c0 = K[b0 - xs], c2 = K[b0 + xs];
  uint32_t n1 = K[b0 + sg * ls], n0 = K[b0 + sg * ls - xs], n2 = K[b0 + sg * ls + xs];
  int ci = b0;                       // the current cell
  int zi = L0 * zls + lane * zxs;    // its z key
  uint32_t kzn = Zk[zi];
  bool any = false;
#pragma unroll 4
  for (int s = 0; s < kFT; ++s) {
    // the line two ahead (the halo line, then the spare row, at the end)
    const int fi = ci + 2 * sg * ls;
    const uint32_t f0 = K[fi - xs], f1 = K[fi], f2 = K[fi + xs];
    const uint32_t kz = kzn;
    kzn = Zk[zi + sg * zls];
    const uint32_t cur = c1;
    const uint32_t mo = min(min(min(c0, c2), min(n0, n1)), min(n2, kKeyMax));  // known a step early
    const uint32_t m = min(min(p0, p1), min(p2, mo));
    const float x = fval(m);
    const float y = x + eps;
    const uint32_t ux = __float_as_uint(x);
    const float xi = y > x ? y : __uint_as_float(x > 0.0f ? ux + 1u : ux - 1u);  // inc_eps(x), x finite
    const uint32_t ki = fkey(xi);
    const uint32_t nk = kz > ki ? kz : ki;
    const bool lower = nk < cur;
    if (lower) {
      const int l = L0 + sg * s;
      const int r = kRows ? l : lane, c = kRows ? lane : l;
      atomicMin(&K[ci], nk);
      atomicOr(&moved[(r * kFT + c) >> 5], 1u << (c & 31));
    }
    any |= lower;
    const uint32_t nc = lower ? nk : cur;  // the cell's key after this step
    // the line just done becomes the previous one, the next the current
    p1 = nc;
    p0 = (uint32_t)__builtin_amdgcn_update_dpp((int)c0, (int)nc, 0x138, 0xF, 0xF, false);  // wave_shr:1
    p2 = (uint32_t)__builtin_amdgcn_update_dpp((int)c2, (int)nc, 0x130, 0xF, 0xF, false);  // wave_shl:1
    c0 = n0;
    c1 = n1;
    c2 = n2;
    n0 = f0;
    n1 = f1;
    n2 = f2;
    ci += sg * ls;
    zi += sg * zls;
  }
  return any;
}

// One round over the queued tiles (FIRST: every tile, with F initialised from
// z in the tile: seeds = z, other valid cells +inf).
template <bool FIRST>
__global__ __launch_bounds__(kFThreads) void k_fill_round(FillArgs a, uint32_t round) {
  // Keys of the tile and its halo ring, and keys of z (kKeyNone: NaN or
  // outside the DEM), each with one spare row before and after, which the
  // sweeps' read-ahead touches at their last step (and then ignores).
  __shared__ uint32_t Kraw[(kFT + 4) * kFK];
  __shared__ uint32_t Zraw[(kFT + 2) * kFZ];
  uint32_t* const K = Kraw + kFK;
  uint32_t* const Zk = Zraw + kFZ;
  __shared__ uint32_t chg[3];
  __shared__ uint32_t sides;
  __shared__ uint32_t moved[kFT * kFT / 32];  // cells lowered during this visit
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t H = a.H, W = a.W;
  if (!FIRST && blockIdx.x == 0 && tid == 0) a.cnt[(round + 2) % 3] = 0;
  const uint32_t n = FIRST ? (uint32_t)(a.TX * a.TY) : a.cnt[round % 3];
  if (n > 0 && blockIdx.x == 0 && tid == 0) atomicMax(&a.cnt[3], round + 1);
  // Tiles are handed out one at a time (visits differ a lot in cost; a
  // static split would wait for the unluckiest workgroup): workgroup b takes
  // entry b first, later ones come from a counter.  Workgroups beyond the
  // queue's length leave without touching the counter.
  __shared__ uint32_t grab;
  if (blockIdx.x == 0 && tid == 0) a.cnt[4 + (round + 2) % 3] = 0;
  for (uint32_t qi = blockIdx.x;;) {
    if (qi >= n) break;
    const uint32_t t = FIRST ? qi : a.queue[round & 1][qi];
    const uint64_t t_start = clock64();
    (void)t_start;
    const int64_t ty = t / a.TX, tx = t - ty * a.TX;
    const int64_t y0 = ty * kFT, x0 = tx * kFT;
    const int th = (int)min((int64_t)kFT, H - y0), tw = (int)min((int64_t)kFT, W - x0);
    if (tid == 0) {
      chg[0] = chg[1] = chg[2] = 0;
      sides = 0;
    }
    if (tid < kFT * kFT / 32) moved[tid] = 0;
    bool known = false;  // any key of the tile or its halo below +inf
    bool anynan = false;  // first round: a NaN (NoData or off the DEM) in the tile or its halo
    {
      float v[kHR], e[kHR];
      load_halo_tile(FIRST ? a.z : a.F, y0, x0, H, W, v, e);
#pragma unroll
      for (int p = 0; p < kHR; ++p) {
        const int r = 4 * p + w;
        if (r >= kFT + 2) continue;
        if (FIRST) {  // raw z bits for the seed test below
          K[r * kFK + lane] = __float_as_uint(v[p]);
          if (lane < 2) K[r * kFK + kFT + lane] = __float_as_uint(e[p]);
          anynan |= __builtin_isnan(v[p]) | ((lane < 2) & __builtin_isnan(e[p]));
        } else {
          K[r * kFK + lane] = __builtin_isnan(v[p]) ? kKeyNone : fkey(v[p]);
          if (lane < 2) K[r * kFK + kFT + lane] = __builtin_isnan(e[p]) ? kKeyNone : fkey(e[p]);
          known |= !__builtin_isnan(v[p]) && v[p] != __builtin_inff();
          known |= !__builtin_isnan(e[p]) && e[p] != __builtin_inff();
        }
      }
    }
    // First round: a whole tile away from the DEM's edges with no NaN in it
    // or its halo ring holds no seed, so every cell starts at +inf and the
    // visit has nothing else to do.
    bool idle = false;
    if (FIRST) {
      const bool nan_near = __syncthreads_or(anynan);
      const bool edge = y0 == 0 || x0 == 0 || y0 + kFT >= H - 1 || x0 + kFT >= W - 1;
      idle = !edge && !nan_near;
    }
    if (idle) {
      float* p0 = a.F + (y0 + w) * W + x0 + lane;
#pragma unroll
      for (int p = 0; p < kTR; ++p) p0[(int64_t)(4 * p) * W] = __builtin_inff();
    } else {
      if (!FIRST) {
        float zv[kTR];
        const bool cx = lane < tw;
        const float* p0 = a.z + (y0 + w) * W + x0 + lane;
#pragma unroll
        for (int p = 0; p < kTR; ++p) zv[p] = (cx && 4 * p + w < th) ? p0[(int64_t)(4 * p) * W] : __builtin_nanf("");
#pragma unroll
        for (int p = 0; p < kTR; ++p) Zk[(4 * p + w) * kFZ + lane] = __builtin_isnan(zv[p]) ? kKeyNone : fkey(zv[p]);
      }
      __syncthreads();
      if (FIRST) {
        // Seeds (valid, on the DEM boundary or next to NaN) start at z, every
        // other valid cell at +inf; the halo ring knows only the DEM-boundary
        // seeds (everything else there is unknown until the next round).
        uint32_t ik[kTR];
#pragma unroll
        for (int p = 0; p < kTR; ++p) {
          const int r = 4 * p + w, c = lane;
          const int h = (r + 1) * kFK + c + 1;
          const float zc = __uint_as_float(K[h]);
          uint32_t key = __builtin_isnan(zc) ? kKeyNone : kKeyInf;
          if (r < th && c < tw && !__builtin_isnan(zc)) {
            const int64_t gy = y0 + r, gx = x0 + c;
            bool seed = gy == 0 || gx == 0 || gy == H - 1 || gx == W - 1;
            seed |= __builtin_isnan(__uint_as_float(K[h + 1])) || __builtin_isnan(__uint_as_float(K[h - 1])) ||
                    __builtin_isnan(__uint_as_float(K[h - kFK - 1])) ||
                    __builtin_isnan(__uint_as_float(K[h - kFK])) ||
                    __builtin_isnan(__uint_as_float(K[h - kFK + 1])) ||
                    __builtin_isnan(__uint_as_float(K[h + kFK - 1])) ||
                    __builtin_isnan(__uint_as_float(K[h + kFK])) || __builtin_isnan(__uint_as_float(K[h + kFK + 1]));
            if (seed) key = fkey(zc);
          }
          ik[p] = key;
          known |= key < kKeyInf;
          Zk[r * kFZ + c] = __builtin_isnan(zc) ? kKeyNone : fkey(zc);
        }
        uint32_t ring[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int j = tid + q * kFThreads;
          ring[q] = kKeyNone;
          if (j < 4 * (kFT + 2) - 4) {
            const int h = ring_index(j);
            const int r = h / kFK, c = h - r * kFK;
            const int64_t gy = y0 - 1 + r, gx = x0 - 1 + c;
            const float v = __uint_as_float(K[h]);
            if (!__builtin_isnan(v)) ring[q] = (gy == 0 || gx == 0 || gy == H - 1 || gx == W - 1) ? fkey(v) : kKeyInf;
            known |= ring[q] < kKeyInf;
          }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kTR; ++p) K[(4 * p + w + 1) * kFK + lane + 1] = ik[p];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int j = tid + q * kFThreads;
          if (j < 4 * (kFT + 2) - 4) K[ring_index(j)] = ring[q];
        }
      }
      // A tile whose cells and halo are all unknown (+inf) cannot change.
      known = __syncthreads_or(known);

      // Directional sweeps: sets until one changes nothing, at most
      // kFillSweepCap + 1 of them.
      const float eps = a.eps;
      bool capped = false;
      int sets = 0;
      for (int it = 0; known; ++it) {
        ++sets;
        if (tid == 0) chg[(it + 1) % 3] = 0;
        bool any;  // this wave lowered a cell
        if (w == 0)
          any = sweep_lines<0>(K, Zk, moved, lane, eps);
        else if (w == 1)
          any = sweep_lines<1>(K, Zk, moved, lane, eps);
        else if (w == 2)
          any = sweep_lines<2>(K, Zk, moved, lane, eps);
        else
          any = sweep_lines<3>(K, Zk, moved, lane, eps);
        if (any) chg[it % 3] = 1;
        __syncthreads();
        if (!chg[it % 3]) break;
        if (it == kFillSweepCap) {  // the tile goes round again
          capped = true;
          break;
        }
      }

      // Write back (first round: everything; later: what moved) and note which
      // neighbours hold a moved cell in their halo.
      uint32_t sb = 0;
      {
        float* p0 = a.F + (y0 + w) * W + x0 + lane;
#pragma unroll 1
        for (int p = 0; p < kTR; ++p) {
          const int r = 4 * p + w, c = lane;
          if (r >= th || c >= tw) continue;
          const uint32_t key = K[(r + 1) * kFK + c + 1];
          float* dst = p0 + (int64_t)(4 * p) * W;
          // first round: every finite value is new to the neighbours
          const bool mv = FIRST ? key < kKeyInf : (moved[(r * kFT + c) >> 5] >> (c & 31)) & 1u;
          if (FIRST) {
            // NoData cells keep their NaN, bit for bit
            *dst = Zk[r * kFZ + c] == kKeyNone ? a.z[(y0 + r) * W + x0 + c] : fval(key);
          } else if (mv) {
            *dst = fval(key);
          }
        }
        // Border cells, one per thread (the row loop above would leave most
        // lanes idle): a neighbouring tile needs another visit only if a moved
        // cell can lower one of its cells; the halo still holds their values
        // from the start of this visit (an upper bound of their current ones).
        if (tid < perim_count(tw, th)) {
          int r, c;
          perim_cell(tid, tw, th, r, c);
          const uint32_t key = K[(r + 1) * kFK + c + 1];
          const bool mv = FIRST ? key < kKeyInf : ((moved[(r * kFT + c) >> 5] >> (c & 31)) & 1u) != 0u;
          if (mv) {
            const uint32_t ki = fkey(inc_eps(fval(key), a.eps));
#pragma unroll
            for (int d = 0; d < 8; ++d) {
              const int dr = d < 3 ? -1 : d < 5 ? 0 : 1;
              const int dc = (d == 0 || d == 3 || d == 5) ? -1 : (d == 1 || d == 6) ? 0 : 1;
              const int rq = r + dr, cq = c + dc;
              if (rq >= 0 && rq < th && cq >= 0 && cq < tw) continue;  // inside this tile
              const uint32_t kq = K[(rq + 1) * kFK + cq + 1];
              if (kq == kKeyNone || kq <= ki) continue;
              const int ny = rq < 0 ? 0 : rq >= th ? 2 : 1, nx = cq < 0 ? 0 : cq >= tw ? 2 : 1;
              sb |= 1u << (ny * 3 + nx);
            }
          }
        }
      }
      if (sb) atomicOr(&sides, sb);
      __syncthreads();
      // The last set still changed something: once more.  (A first-round tile
      // whose halo guess was too high is queued by the neighbour that knows
      // better.)
      if (capped && tid == 0) fill_enqueue(a, t, round + 1);
      if (tid < 9 && tid != 4) {
        // bit 3*(dy+1) + (dx+1): the neighbouring tile at (dy, dx)
        const int64_t ny = ty + tid / 3 - 1, nx = tx + tid % 3 - 1;
        if ((sides >> tid) & 1u && ny >= 0 && ny < a.TY && nx >= 0 && nx < a.TX)
          fill_enqueue(a, (uint32_t)(ny * a.TX + nx), round + 1);
      }
      D8_FILL_STAT(round, sets, t_start);
    }  // not an idle first-round tile
    if (tid == 0) grab = gridDim.x + atomicAdd(&a.cnt[4 + round % 3], 1u);
    __syncthreads();  // also: LDS is reused by the next tile
    qi = grab;
    __syncthreads();  // every thread has read grab before it is written again
  }
}

__global__ void k_fill_reset(FillArgs a) {
  const int64_t nt = a.TX * a.TY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x)
    a.qround[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 8) a.cnt[threadIdx.x] = 0;
}

}  // namespace

// As many workgroups as the chip holds at once (they then pull tiles from
// the counter), never more than there are tiles.
template <bool FIRST>
static int fill_grid_blocks(int64_t ntiles) {
  static std::atomic<int> per_chip[64];  // per device, 0 until queried (the same value from any thread)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int n = per_chip[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fill_round<FIRST>, kFThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
        cus <= 0) {
      per_cu = 4;
      cus = 256;
    }
    n = per_cu * cus;
    per_chip[dev].store(n, std::memory_order_relaxed);
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, n));
}

hipError_t launch_fill_reset(const FillArgs& a, hipStream_t s) {
  const int64_t nt = a.TX * a.TY;
  const int g = (int)std::min<int64_t>((nt + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_reset, dim3(std::max(g, 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_round(const FillArgs& a, uint32_t round, hipStream_t s) {
  if (round == 0)
    hipLaunchKernelGGL(k_fill_round<true>, dim3(fill_grid_blocks<true>(a.TX * a.TY)), dim3(kFThreads), 0, s, a,
                       round);
  else
    hipLaunchKernelGGL(k_fill_round<false>, dim3(fill_grid_blocks<false>(a.TX * a.TY)), dim3(kFThreads), 0, s,
                       a, round);
  return hipGetLastError();
}

}  // namespace d8
