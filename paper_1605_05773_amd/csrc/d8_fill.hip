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
// idea as the accumulation: a tile relaxes to its own fixed point given the
// current values of its one-cell halo, writes back what changed and, when a
// perimeter cell changed, queues the neighbouring tiles whose halo holds that
// cell for the next round.  Rounds repeat until no tile is queued.
//
// Inside a tile the four waves of the workgroup sweep concurrently in the four
// axis directions (rows down, rows up, columns right, columns left; one cell
// per lane per step), so values travel up to 64 cells along any monotone
// run per sweep.  Updates lower a cell's key with an LDS atomic min, which
// keeps every value an upper bound of the fixed point while the waves race.
// A cell already at z is final (values only fall and never below z), so
// seeds and undisturbed terrain cost two LDS reads per visit.
#include <algorithm>

#include "d8_internal.hpp"

namespace d8 {
namespace {

constexpr int kFT = 64;            // tile side
constexpr int kFK = kFT + 3;       // row stride of the key array (halo ring + 1 pad: odd)
constexpr int kFZ = kFT + 1;       // row stride of the elevation array (odd)
constexpr int kFThreads = 256;     // four waves
constexpr uint32_t kKeyInf = 0xFF800000u;  // key of +inf: also "no value" (outside, NaN)
constexpr int kFillSweepCap = 255;         // sweep sets per tile visit

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

__device__ __forceinline__ void fill_enqueue(const FillArgs& a, uint32_t t, uint32_t next_round) {
  if (atomicMax(&a.qround[t], next_round) < next_round) {
    const uint32_t slot = atomicAdd(&a.cnt[next_round % 3], 1u);
    a.queue[next_round & 1][slot] = t;
  }
}

// One round over the queued tiles (FIRST: every tile, with F initialised from
// z in the tile: seeds = z, other valid cells +inf).
template <bool FIRST>
__global__ __launch_bounds__(kFThreads) void k_fill_round(FillArgs a, uint32_t round) {
  __shared__ uint32_t K[(kFT + 2) * kFK];
  __shared__ float Z[kFT * kFZ];
  __shared__ uint32_t chg[3];
  __shared__ uint32_t sides;
  const int tid = threadIdx.x;
  const int64_t H = a.H, W = a.W;
  if (!FIRST && blockIdx.x == 0 && tid == 0) a.cnt[(round + 2) % 3] = 0;
  const uint32_t n = FIRST ? (uint32_t)(a.TX * a.TY) : a.cnt[round % 3];
  if (n > 0 && blockIdx.x == 0 && tid == 0) atomicMax(&a.cnt[3], round + 1);
  constexpr int KPT = kFT * kFT / kFThreads;
  for (uint32_t qi = blockIdx.x; qi < n; qi += gridDim.x) {
    const uint32_t t = FIRST ? qi : a.queue[round & 1][qi];
    const int64_t ty = t / a.TX, tx = t - ty * a.TX;
    const int64_t y0 = ty * kFT, x0 = tx * kFT;
    const int th = (int)min((int64_t)kFT, H - y0), tw = (int)min((int64_t)kFT, W - x0);
    uint32_t ik[KPT];  // keys at entry (change detection)
    if (tid == 0) {
      chg[0] = chg[1] = chg[2] = 0;
      sides = 0;
    }
    if (FIRST) {
      // z with its one-cell halo, as raw bits (NaN outside the DEM)
      for (int i = tid; i < (kFT + 2) * (kFT + 2); i += kFThreads) {
        const int r = i / (kFT + 2), c = i - r * (kFT + 2);
        const int64_t gy = y0 - 1 + r, gx = x0 - 1 + c;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        K[r * kFK + c] = in ? __float_as_uint(a.z[gy * W + gx]) : 0x7FC00000u;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int i = tid + k * kFThreads;
        const int r = i / kFT, c = i - r * kFT;
        const int h = (r + 1) * kFK + c + 1;
        const float zc = __uint_as_float(K[h]);
        uint32_t key = kKeyInf;
        if (r < th && c < tw && !__builtin_isnan(zc)) {
          const int64_t gy = y0 + r, gx = x0 + c;
          bool seed = gy == 0 || gx == 0 || gy == H - 1 || gx == W - 1;
          if (!seed) {
            const int nb[8] = {1, 1 - kFK, -kFK, -kFK - 1, -1, kFK - 1, kFK, kFK + 1};
#pragma unroll
            for (int d = 0; d < 8; ++d) seed |= __builtin_isnan(__uint_as_float(K[h + nb[d]]));
          }
          if (seed) key = fkey(zc);
        }
        ik[k] = key;
        Z[r * kFZ + c] = zc;
      }
      // halo ring: DEM-boundary cells are seeds; everything else is unknown
      uint32_t ring[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = tid + q * kFThreads;
        ring[q] = kKeyInf;
        if (j < 4 * (kFT + 2) - 4) {
          int r, c;
          if (j < kFT + 2) { r = 0; c = j; }
          else if (j < 2 * (kFT + 2)) { r = kFT + 1; c = j - (kFT + 2); }
          else if (j < 3 * (kFT + 2) - 2) { r = j - 2 * (kFT + 2) + 1; c = 0; }
          else { r = j - 3 * (kFT + 2) + 3; c = kFT + 1; }
          const int64_t gy = y0 - 1 + r, gx = x0 - 1 + c;
          const float v = __uint_as_float(K[r * kFK + c]);
          if (!__builtin_isnan(v) && (gy == 0 || gx == 0 || gy == H - 1 || gx == W - 1)) ring[q] = fkey(v);
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int i = tid + k * kFThreads;
        K[(i / kFT + 1) * kFK + i % kFT + 1] = ik[k];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = tid + q * kFThreads;
        if (j < 4 * (kFT + 2) - 4) {
          int r, c;
          if (j < kFT + 2) { r = 0; c = j; }
          else if (j < 2 * (kFT + 2)) { r = kFT + 1; c = j - (kFT + 2); }
          else if (j < 3 * (kFT + 2) - 2) { r = j - 2 * (kFT + 2) + 1; c = 0; }
          else { r = j - 3 * (kFT + 2) + 3; c = kFT + 1; }
          K[r * kFK + c] = ring[q];
        }
      }
    } else {
      for (int i = tid; i < (kFT + 2) * (kFT + 2); i += kFThreads) {
        const int r = i / (kFT + 2), c = i - r * (kFT + 2);
        const int64_t gy = y0 - 1 + r, gx = x0 - 1 + c;
        uint32_t key = kKeyInf;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
          const float f = a.F[gy * W + gx];
          if (!__builtin_isnan(f)) key = fkey(f);
        }
        K[r * kFK + c] = key;
      }
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int i = tid + k * kFThreads;
        const int r = i / kFT, c = i - r * kFT;
        Z[r * kFZ + c] = (r < th && c < tw) ? a.z[(y0 + r) * W + x0 + c] : __builtin_nanf("");
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const int i = tid + k * kFThreads;
        ik[k] = K[(i / kFT + 1) * kFK + i % kFT + 1];
      }
    }
    __syncthreads();

    // Directional sweeps until a full set of them changes nothing.
    const int w = tid >> 6, lane = tid & 63;
    const float eps = a.eps;
    bool capped = false;
    for (int it = 0;; ++it) {
      if (tid == 0) chg[(it + 1) % 3] = 0;
      bool any = false;
      for (int s = 0; s < kFT; ++s) {
        const int r = w == 0 ? s : w == 1 ? kFT - 1 - s : lane;
        const int c = w == 2 ? s : w == 3 ? kFT - 1 - s : lane;
        if (r < th && c < tw) {
          const float zc = Z[r * kFZ + c];
          const int h = (r + 1) * kFK + c + 1;
          const uint32_t cur = K[h];
          const uint32_t kz = fkey(zc);
          if (!__builtin_isnan(zc) && cur != kz) {
            uint32_t m = min(min(K[h - kFK - 1], K[h - kFK]), min(K[h - kFK + 1], K[h - 1]));
            m = min(m, min(min(K[h + 1], K[h + kFK - 1]), min(K[h + kFK], K[h + kFK + 1])));
            const uint32_t ki = fkey(inc_eps(fval(m), eps));
            const uint32_t nk = kz > ki ? kz : ki;
            if (nk < cur) {
              atomicMin(&K[h], nk);
              any = true;
            }
          }
        }
      }
      if (any) chg[it % 3] = 1;
      __syncthreads();
      if (!chg[it % 3]) break;
      if (it == kFillSweepCap) {  // bounded work per visit: the tile goes round again
        capped = true;
        break;
      }
    }

    // Write back what changed; note which neighbours see a changed cell.
    uint32_t sb = 0;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int i = tid + k * kFThreads;
      const int r = i / kFT, c = i - r * kFT;
      if (r >= th || c >= tw) continue;
      const uint32_t key = K[(r + 1) * kFK + c + 1];
      const int64_t g = (y0 + r) * W + x0 + c;
      if (FIRST) {
        a.F[g] = __builtin_isnan(Z[r * kFZ + c]) ? Z[r * kFZ + c] : fval(key);
      } else if (key != ik[k]) {
        a.F[g] = fval(key);
        const bool n_ = r == 0, s_ = r == th - 1, w_ = c == 0, e_ = c == tw - 1;
        sb |= (n_ ? 1u : 0u) | (s_ ? 2u : 0u) | (w_ ? 4u : 0u) | (e_ ? 8u : 0u) |
              (n_ && w_ ? 16u : 0u) | (n_ && e_ ? 32u : 0u) | (s_ && w_ ? 64u : 0u) | (s_ && e_ ? 128u : 0u);
      }
    }
    if (!FIRST && sb) atomicOr(&sides, sb);
    __syncthreads();
    if (FIRST || capped) {
      // the halo was a guess, or the sweeps stopped early: once more
      if (tid == 0) fill_enqueue(a, t, round + 1);
    }
    if (!FIRST && tid < 8) {
      const uint32_t bits = sides;
      const int dy[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
      const int dx[8] = {0, 0, -1, 1, -1, 1, -1, 1};
      const int64_t ny = ty + dy[tid], nx = tx + dx[tid];
      if ((bits >> tid) & 1u && ny >= 0 && ny < a.TY && nx >= 0 && nx < a.TX)
        fill_enqueue(a, (uint32_t)(ny * a.TX + nx), round + 1);
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

__global__ void k_fill_reset(FillArgs a) {
  const int64_t nt = a.TX * a.TY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x)
    a.qround[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 4) a.cnt[threadIdx.x] = 0;
}

}  // namespace

static int fill_grid_blocks(int64_t ntiles) {
  // four 34 KB workgroups fit one CU's LDS; one wave of them covers the chip
  return (int)std::min<int64_t>(ntiles, 256 * 4);
}

hipError_t launch_fill_reset(const FillArgs& a, hipStream_t s) {
  const int64_t nt = a.TX * a.TY;
  const int g = (int)std::min<int64_t>((nt + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_reset, dim3(std::max(g, 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_round(const FillArgs& a, uint32_t round, hipStream_t s) {
  const int g = fill_grid_blocks(a.TX * a.TY);
  if (round == 0)
    hipLaunchKernelGGL(k_fill_round<true>, dim3(g), dim3(kFThreads), 0, s, a, round);
  else
    hipLaunchKernelGGL(k_fill_round<false>, dim3(g), dim3(kFThreads), 0, s, a, round);
  return hipGetLastError();
}

}  // namespace d8
