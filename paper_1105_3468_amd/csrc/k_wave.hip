// Wavefront sweeps for factors with the structure of a 2D grid: every row
// k = j * nx + i of a lower factor depends at most on k - 1 (same grid row,
// i > 0) and k - nx (previous grid row).  ILU(0) of a five-point operator in
// natural order has exactly this structure; an upper factor (k + 1, k + nx)
// is a lower factor of the reversed grid.
//
// The general sweep pays one dependency level (a publish-and-poll hop) per
// anti-diagonal of the grid.  Here a wave owns 64 grid rows, one per lane,
// and walks them with a skew of one column per lane: at step s lane l treats
// column i = s - l of grid row j = 64 w + l.  Both dependencies are then
// results of the previous step, the left one in the lane's own register and
// the one below in lane l - 1, moved over with a DPP lane shift; only lane 0
// reads the previous wave's lane 63, through memory (value-as-flag, like the
// general sweep).  A step costs a few vector instructions instead of a hop,
// and wave w runs about 64 steps behind wave w - 1.
//
// Positions p = (w * S + s) * 64 + l (S = nx + 63 steps per wave) hold the
// operands of step s of lane l, so every step reads and writes one contiguous
// 64-element segment; positions outside the grid hold zero coefficients and
// a zero right-hand side, which make their results zero.  The positions of
// an upper factor are those of the lower layout read backwards, so the upper
// sweep reads the lower sweep's output (its right-hand side) at total - 1 - p
// without any reordering in between.  Terms are added in ascending column
// order with the same fused multiply-adds as the general sweep, so the
// results are bitwise identical to it.
#include <algorithm>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int WAVE_PF = 8;  // steps of operands in flight

// Lane l receives lane l - 1's value (lane 0 receives 0): DPP wave_shr:1.
__device__ __forceinline__ int lane_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float lane_shr1(float v) {
  return __builtin_bit_cast(float, lane_shr1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_shr1(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)lane_shr1((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)lane_shr1((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <class T>
struct Pair;
template <>
struct Pair<double> { using type = double2; };
template <>
struct Pair<float> { using type = float2; };

// coef[p] = (coefficient of the neighbour below, coefficient of the left
// neighbour); UP_FIRST: the neighbour below has the smaller original column
// (lower factors), else the left one (upper factors).
template <class T, bool DIAG, bool UP_FIRST, bool REV>
__global__ __launch_bounds__(64) void k_wave(int S, int nx, int64_t total, const typename Pair<T>::type* __restrict__ coef,
                                             const T* __restrict__ dinv, T* rhs, T* out, int* abort_flag,
                                             uint64_t limit) {
  const int w = blockIdx.x, l = threadIdx.x;
  const int64_t p0 = (int64_t)w * S * 64 + l;
  // previous wave, lane 63, step s + 63 (the same column as lane 0, step s)
  const T* prev = out + ((int64_t)(w - 1) * S + 63) * 64 + 63;
  const bool reads_prev = l == 0 && w > 0;
  T cu[WAVE_PF], cl[WAVE_PF], b[WAVE_PF], d[WAVE_PF], x[WAVE_PF];
  auto fetch = [&](int s, int u) {
    const int64_t p = p0 + (int64_t)std::min(s, S - 1) * 64;
    const typename Pair<T>::type c = coef[p];
    cu[u] = c.x;
    cl[u] = c.y;
    b[u] = REV ? rhs[total - 1 - p] : rhs[p];
    d[u] = DIAG ? dinv[p] : (T)1;
    x[u] = (reads_prev && s < nx) ? ld_agent(prev + (int64_t)s * 64) : (T)0;
  };
#pragma unroll
  for (int u = 0; u < WAVE_PF; ++u) fetch(u, u);
  T yp = (T)0;  // this lane's result of the previous step
  for (int s0 = 0; s0 < S; s0 += WAVE_PF) {
#pragma unroll
    for (int u = 0; u < WAVE_PF; ++u) {
      const int s = s0 + u;
      if (s >= S) break;
      T xb = x[u];
      if (reads_prev && s < nx && is_sentinel(xb)) {
        const uint64_t t0 = wall_clock64();
        unsigned it = 0;
#pragma clang loop unroll(disable)
        do {
          __builtin_amdgcn_s_sleep(1);
          xb = ld_agent(prev + (int64_t)s * 64);
          if (is_sentinel(xb) && (++it & 63u) == 0) {
            if (ld_agent(abort_flag)) { xb = (T)__builtin_nan(""); break; }
            if (wall_clock64() - t0 > limit) {
              st_agent(abort_flag, 1);
              xb = (T)__builtin_nan("");
              break;
            }
          }
        } while (is_sentinel(xb));
      }
      T up = lane_shr1(yp);
      if (l == 0) up = xb;
      T acc = (T)0;
      if (UP_FIRST) {
        acc += cu[u] * up;
        acc += cl[u] * yp;
      } else {
        acc += cl[u] * yp;
        acc += cu[u] * up;
      }
      T y = b[u] - acc;
      if (DIAG) y *= d[u];
      if (is_sentinel(y)) y = (T)__builtin_nan("");
      const int64_t p = p0 + (int64_t)s * 64;
      st_agent(out + p, y);
      if (REV) rhs[total - 1 - p] = sentinel_of<T>(0);
      yp = y;
      fetch(s + WAVE_PF, u);
    }
  }
}

// positions of the lower layout -> cell (or -1 outside the grid)
__device__ __forceinline__ int wave_cell(int64_t q, int S, int nx, int ny) {
  const int l = (int)(q & 63);
  const int64_t ws = q >> 6;
  const int w = (int)(ws / S), s = (int)(ws - (int64_t)w * S);
  const int j = 64 * w + l, i = s - l;
  return (i >= 0 && i < nx && j < ny) ? j * nx + i : -1;
}

template <class T, class TR>
__global__ void k_wave_gather(int64_t total, int S, int nx, int ny, const TR* __restrict__ z, T* __restrict__ zs) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = wave_cell(p, S, nx, ny);
    zs[p] = c >= 0 ? (T)z[c] : (T)0;
  }
}

// out[cell] = ts[p] for the upper layout (cell of lower position total-1-p);
// ts is reset to the sentinel for the next sweep
template <class T>
__global__ void k_wave_scatter(int64_t total, int S, int nx, int ny, T* __restrict__ ts, T* __restrict__ t) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = wave_cell(total - 1 - p, S, nx, ny);
    if (c >= 0) t[c] = ts[p];
    ts[p] = sentinel_of<T>(0);
  }
}

static uint64_t wave_limit_ticks() {
  static uint64_t ticks = 0;
  if (!ticks) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
      (void)hipGetLastError();
      khz = 100000;
    }
    ticks = (uint64_t)khz * 1000ull * 4ull;  // 4 seconds
  }
  return ticks;
}

template <class T>
void launch_wave_pair(const WaveGrid& g, const WaveSweep& lo, const WaveSweep& up, const void* z, bool z_f64, T* zs,
                      T* ys, T* ts, T* t, int* abort_flag, hipStream_t s) {
  constexpr bool F32 = sizeof(T) == 4;
  using P2 = typename Pair<T>::type;
  const unsigned gb = (unsigned)std::min<int64_t>(4096, (g.total + 255) / 256);
  if (z_f64)
    hipLaunchKernelGGL((k_wave_gather<T, double>), dim3(gb), dim3(256), 0, s, g.total, g.S, g.nx, g.ny,
                       (const double*)z, zs);
  else
    hipLaunchKernelGGL((k_wave_gather<T, T>), dim3(gb), dim3(256), 0, s, g.total, g.S, g.nx, g.ny, (const T*)z, zs);
  const uint64_t lim = wave_limit_ticks();
  auto co = [&](const WaveSweep& f) { return F32 ? (const P2*)f.coef32.p : (const P2*)f.coef.p; };
  auto di = [&](const WaveSweep& f) { return F32 ? (const T*)f.dinv32.p : (const T*)f.dinv.p; };
  // lower factor: neighbour below first; upper factor: left neighbour first,
  // right-hand side = the lower sweep's output read backwards
  if (lo.has_diag)
    hipLaunchKernelGGL((k_wave<T, true, true, false>), dim3(g.W), dim3(64), 0, s, g.S, g.nx, g.total, co(lo), di(lo),
                       zs, ys, abort_flag, lim);
  else
    hipLaunchKernelGGL((k_wave<T, false, true, false>), dim3(g.W), dim3(64), 0, s, g.S, g.nx, g.total, co(lo),
                       di(lo), zs, ys, abort_flag, lim);
  if (up.has_diag)
    hipLaunchKernelGGL((k_wave<T, true, false, true>), dim3(g.W), dim3(64), 0, s, g.S, g.nx, g.total, co(up), di(up),
                       ys, ts, abort_flag, lim);
  else
    hipLaunchKernelGGL((k_wave<T, false, false, true>), dim3(g.W), dim3(64), 0, s, g.S, g.nx, g.total, co(up),
                       di(up), ys, ts, abort_flag, lim);
  hipLaunchKernelGGL((k_wave_scatter<T>), dim3(gb), dim3(256), 0, s, g.total, g.S, g.nx, g.ny, ts, t);
  HIPCK(hipGetLastError());
}
template void launch_wave_pair<double>(const WaveGrid&, const WaveSweep&, const WaveSweep&, const void*, bool,
                                       double*, double*, double*, double*, int*, hipStream_t);
template void launch_wave_pair<float>(const WaveGrid&, const WaveSweep&, const WaveSweep&, const void*, bool,
                                      float*, float*, float*, float*, int*, hipStream_t);

}  // namespace gmg
