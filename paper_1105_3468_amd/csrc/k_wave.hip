// Wavefront sweeps for factors with the structure of a 2D grid (below) or
// of a 3D grid (k_wave3, further down).  2D: every row k = j * nx + i of a
// lower factor depends at most on k - 1 (same grid row, i > 0) and k - nx
// (previous grid row).  ILU(0) of a five-point operator in natural order has
// exactly this structure; an upper factor (k + 1, k + nx) is a lower factor
// of the reversed grid.
//
// The general sweep pays one dependency level (a publish-and-poll hop) per
// anti-diagonal of the grid.  Here a wave owns 64 grid rows, one per lane,
// and walks them with a skew of one column per lane: at step s lane l treats
// column i = s - l of grid row j = 64 w + l.  Both dependencies are then
// results of the previous step, the left one in the lane's own register and
// the one below in lane l - 1, moved over with a DPP lane shift; only lane 0
// reads the previous wave's lane 63, through memory (value-as-flag, like the
// general sweep).  A step costs a few vector instructions instead of a hop,
// and wave w runs about 64 steps behind wave w - 1.  So that the computing
// wave never waits on memory latency, two more waves of its workgroup stream
// its operands into an LDS ring ahead of it.
//
// Positions p = (w * S + s) * 64 + l (S = nx + 63 steps per wave, rounded up
// to whole pairs of chunks of the kernel below) hold the
// operands of step s of lane l, so every step reads and writes one contiguous
// 64-element segment; positions outside the grid hold zero coefficients and
// a zero right-hand side, which make their results zero.  The positions of
// an upper factor are those of the lower layout read backwards, so the upper
// sweep reads the lower sweep's output (its right-hand side) at total - 1 - p
// without any reordering in between.  Terms are added in ascending column
// order with the same fused multiply-adds as the general sweep, so the
// results are bitwise identical to it.
#include <algorithm>
#include <type_traits>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

// One workgroup per 64 grid rows: wave 0 computes; waves 1 .. WAVE_PRODUCERS
// stream the operands of chunks of WAVE_CH steps into an LDS ring of
// WAVE_SLOTS chunks (producer k takes chunks k, k + P, k + 2P, ..., each
// keeping WAVE_D chunks of loads in flight) and flag each chunk ready; the
// last wave polls the previous band's boundary values into a second ring of
// WAVE_XRING steps.  The computing wave thus issues no global loads: its
// stores, which share the in-order memory counter with loads, never hold it
// up.  Its step is a handful of instructions (a wave issues at most one per
// four cycles), so everything else is moved off it: ring offsets are taken
// once per chunk, and the producers screen the right-hand side for the
// not-yet-computed marker (a NaN carrying the marker's payload becomes a plain
// NaN), so that no result can carry the marker and results are published
// without a test.
constexpr int WAVE_CH = 8;
constexpr int WAVE_D = 2;
constexpr int WAVE_SLOTS = 6;
constexpr int WAVE_RING = WAVE_CH * WAVE_SLOTS;
constexpr int WAVE_PRODUCERS = 4;
constexpr int WAVE_XRING = 256;
constexpr int WAVE_THREADS = 64 * (2 + WAVE_PRODUCERS);
static_assert(WAVE_XRING % WAVE_CH == 0, "a chunk's boundary values must not wrap around the ring");

// Lane l receives lane l - 1's value v; lane 0 keeps lane0 (DPP wave_shr:1
// without bound control leaves the destination of a lane with no source).
__device__ __forceinline__ int lane_shr1(int lane0, int v) {
  return __builtin_amdgcn_update_dpp(lane0, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ float lane_shr1(float lane0, float v) {
  return __builtin_bit_cast(float, lane_shr1(__builtin_bit_cast(int, lane0), __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_shr1(double lane0, double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v), o = __builtin_bit_cast(uint64_t, lane0);
  const uint32_t lo = (uint32_t)lane_shr1((int)(uint32_t)o, (int)(uint32_t)b);
  const uint32_t hi = (uint32_t)lane_shr1((int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <class T>
struct Pair;
template <>
struct Pair<double> { using type = double2; };
template <>
struct Pair<float> { using type = float2; };

// one step's operands of one lane in the LDS ring: the two coefficients, the
// right-hand side and the reciprocal diagonal (two 16-byte LDS reads for FP64)
template <class T>
struct alignas(4 * sizeof(T)) WaveOp {
  T cb, cl, b, d;  // coefficient of the neighbour below, of the left one
};

// Bounded wait on an LDS progress counter (relaxed loads); false when the
// sweep is abandoned (abort flag raised, or the time limit hit here).  SLEEP:
// back off between polls (producers ahead of the consumer must not flood the
// LDS pipe the consumer reads its operands through).  READ_ABORT: also poll
// the abort flag; the computing wave does not (a global load on its path
// makes the compiler wait for all of its outstanding stores where the load's
// register is reused), so it gives up on its own time limit only.
template <int SLEEP, bool READ_ABORT = true>
__device__ __forceinline__ bool wait_lds_at_least(const int* ctr, int want, int* abort_flag, uint64_t limit) {
  if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= want) return true;
  const uint64_t t0 = wall_clock64();
  unsigned it = 0;
#pragma clang loop unroll(disable)
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < want) {
    __builtin_amdgcn_s_sleep(SLEEP);
    if ((++it & 255u) == 0) {
      if (READ_ABORT && ld_agent(abort_flag)) return false;
      if (wall_clock64() - t0 > limit) {
        st_agent(abort_flag, 1);
        return false;
      }
    }
  }
  return true;
}

// Bounded wait for an LDS flag to equal `want` (the computing wave: relaxed
// loads, no sleep, no global load on its path); false when abandoned.
__device__ __forceinline__ bool wait_lds_equal(const int* flag, int want, int* abort_flag, uint64_t limit) {
  const uint64_t t0 = wall_clock64();
  unsigned it = 0;
#pragma clang loop unroll(disable)
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != want) {
    if ((++it & 255u) == 0 && wall_clock64() - t0 > limit) {
      st_agent(abort_flag, 1);
      return false;
    }
  }
  return true;
}

// LDS-only release / acquire: orders the ring's data against its counters
// without waiting for global memory operations.
__device__ __forceinline__ void lds_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local"); }
__device__ __forceinline__ void lds_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local"); }

// coef[p] = (coefficient of the neighbour below, coefficient of the left
// neighbour); UP_FIRST: the neighbour below has the smaller original column
// (lower factors), else the left one (upper factors).  REV: the right-hand
// side is read at total - 1 - p.
//
// nb > 1 sweeps nb right-hand sides in one launch: workgroup w * nb + r runs
// band w of column r, whose right-hand side and output are the position
// layouts at rhs + r * total and out + r * total.  A band waits only on the
// band before it in the same column, which has the lower workgroup index, so
// the launch drains as with one column.
template <class T, bool DIAG, bool UP_FIRST, bool REV>
__global__ __launch_bounds__(WAVE_THREADS) void k_wave(int S, int nx, int64_t total,
                                                       const typename Pair<T>::type* __restrict__ coef,
                                                       const T* __restrict__ dinv, const T* __restrict__ rhs, T* out,
                                                       int* abort_flag, uint64_t limit, int nb) {
  using P2 = typename Pair<T>::type;
  __shared__ WaveOp<T> r_op[WAVE_RING][64];
  __shared__ T r_x[WAVE_XRING];      // previous band's boundary values
  __shared__ int ready[WAVE_SLOTS];  // chunk c + 1 once chunk c is in its slot c % WAVE_SLOTS
  __shared__ int xready;             // boundary values in r_x
  __shared__ int consumed;           // steps finished by the consumer
  // the role is the same for the whole wave: taken from lane 0 so the role
  // branches are scalar and no role's pending loads reach another's code
  const int w = blockIdx.x / nb, l = threadIdx.x & 63, role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  {
    const int col = blockIdx.x - w * nb;
    rhs += (int64_t)col * total;
    out += (int64_t)col * total;
  }
  const int64_t p0 = (int64_t)w * S * 64 + l;
  const int nchunks = S / WAVE_CH;
  if (threadIdx.x < WAVE_SLOTS) ready[threadIdx.x] = 0;
  if (threadIdx.x == 0) { consumed = 0; xready = 0; }
  // the boundary ring starts at zero: the consumer reads it for every step,
  // and steps without a boundary value (first band, padding) have a zero
  // coefficient for it, which a finite value times zero leaves exact
  for (int i = threadIdx.x; i < WAVE_XRING; i += WAVE_THREADS) r_x[i] = (T)0;
  __syncthreads();

  // boundary values exist for steps s < xn (the previous band's lane 63 at
  // step s + 63); later steps are padding
  const int xn = S - 63;
  if (role == 1 + WAVE_PRODUCERS) {
    // ------------------------------------------- previous band's boundary
    if (w == 0) return;
    const T* prev = out + ((int64_t)(w - 1) * S + 63) * 64 + 63;
    int next = 0;
    const uint64_t t0 = wall_clock64();
    unsigned it = 0;
#pragma clang loop unroll(disable)
    while (next < xn) {
      // ring space: slots of steps next .. next + 63 were used WAVE_XRING steps earlier
      if (!wait_lds_at_least<4>(&consumed, next + 64 - WAVE_XRING, abort_flag, limit)) return;
      const int s = next + l;
      const T v = s < xn ? ld_agent(prev + (int64_t)s * 64) : (T)0;
      const uint64_t pend = __ballot(s < xn && is_sentinel(v));
      const int k = pend ? (int)__builtin_ctzll(pend) : 64;  // leading published steps
      if (k > 0) {
        if (l < k) r_x[s % WAVE_XRING] = v;
        lds_release();
        next = std::min(next + k, xn);
        if (l == 0) __hip_atomic_store(&xready, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        __builtin_amdgcn_s_sleep(1);
        if ((++it & 63u) == 0) {
          if (ld_agent(abort_flag)) return;
          if (wall_clock64() - t0 > limit) {
            st_agent(abort_flag, 1);
            return;
          }
        }
      }
    }
    return;
  }

  if (role > 0) {
    // ---------------------------------------------------------- producer
    const int k = role - 1;
    P2 rc[WAVE_D][WAVE_CH];
    T rb[WAVE_D][WAVE_CH], rd[WAVE_D][WAVE_CH];
    auto issue = [&](int c, int slot) {
#pragma unroll
      for (int u = 0; u < WAVE_CH; ++u) {
        const int64_t p = p0 + (int64_t)(c * WAVE_CH + u) * 64;
        rc[slot][u] = coef[p];
        rb[slot][u] = REV ? rhs[total - 1 - p] : rhs[p];
        if (DIAG) rd[slot][u] = dinv[p];
      }
    };
    // chunks of this producer: c = k, k + P, k + 2P, ...; the d-th of them
    // uses register slot d % WAVE_D
#pragma unroll
    for (int d = 0; d < WAVE_D; ++d) {
      const int c = k + d * WAVE_PRODUCERS;
      if (c < nchunks) issue(c, d);
    }
    for (int d0 = 0;; d0 += WAVE_D) {
#pragma unroll
      for (int dd = 0; dd < WAVE_D; ++dd) {
        const int c = k + (d0 + dd) * WAVE_PRODUCERS;
        if (c >= nchunks) return;
        // the ring slot of chunk c last held chunk c - WAVE_SLOTS
        if (!wait_lds_at_least<4>(&consumed, (c + 1 - WAVE_SLOTS) * WAVE_CH, abort_flag, limit)) return;
        const int rb0 = (c % WAVE_SLOTS) * WAVE_CH;
#pragma unroll
        for (int u = 0; u < WAVE_CH; ++u) {
          WaveOp<T> op;
          op.cb = rc[dd][u].x;
          op.cl = rc[dd][u].y;
          op.b = is_sentinel(rb[dd][u]) ? (T)__builtin_nan("") : rb[dd][u];
          op.d = DIAG ? rd[dd][u] : (T)1;
          r_op[rb0 + u][l] = op;
        }
        lds_release();
        if (l == 0) __hip_atomic_store(&ready[c % WAVE_SLOTS], c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int cn = c + WAVE_D * WAVE_PRODUCERS;
        if (cn < nchunks) issue(cn, dd);
      }
    }
  }

  // ------------------------------------------------------------ consumer
  // Chunks of WAVE_CH steps, two at a time (S is a multiple of 2 WAVE_CH):
  // set A holds the operands of the even chunk, set B of the odd one, each
  // read from the ring while the other set computes, so no values are moved
  // between registers.  A wait that is abandoned (abort flag, time limit)
  // only marks the sweep dead: the rest runs without waiting and its results
  // are discarded by the host, so the loop has no early exit.
  const bool reads_prev = w > 0;
  bool live = true;
  int seen_x = 0;
  WaveOp<T> opA[WAVE_CH], opB[WAVE_CH];
  T xA[WAVE_CH], xB[WAVE_CH];
  // The ready flag of a chunk is read one chunk ahead, while the chunk before
  // it computes, so its value is at hand (the LDS wait at the end of every
  // chunk covers it) when the chunk's operands are read; only a chunk that
  // was not ready then is waited for.
  auto flag_of = [&](int c) {
    return c < nchunks ? __hip_atomic_load(&ready[c % WAVE_SLOTS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                       : 0;
  };
  // make sure chunk c and its boundary values are in LDS (seen: its ready
  // flag as read earlier), then read its operands (ring offsets fixed per
  // chunk: the reads take immediate offsets)
  auto take = [&](int c, int seen, WaveOp<T>(&op)[WAVE_CH], T(&xv)[WAVE_CH]) {
    const int slot = c % WAVE_SLOTS;
    if (live && seen != c + 1) live = wait_lds_equal(&ready[slot], c + 1, abort_flag, limit);
    const int s0 = c * WAVE_CH;
    if (reads_prev && s0 < xn) {
      const int need = std::min(s0 + WAVE_CH, xn);
      if (live && seen_x < need) {
        seen_x = __hip_atomic_load(&xready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (seen_x < need) {
          live = wait_lds_at_least<0, false>(&xready, need, abort_flag, limit);
          seen_x = need;
        }
      }
    }
    lds_acquire();
    const int r0 = slot * WAVE_CH;
    const T* rx = r_x + s0 % WAVE_XRING;
#pragma unroll
    for (int u = 0; u < WAVE_CH; ++u) {
      op[u] = r_op[r0 + u][l];
      xv[u] = rx[u];
    }
  };
  T yp = (T)0;  // this lane's result of the previous step
  // the steps of chunk c; results stored with immediate offsets from one
  // base, each one step later in program order so that its store fills the
  // latency of the next step's chain instead of lengthening it
  auto run = [&](int c, const WaveOp<T>(&op)[WAVE_CH], const T(&xv)[WAVE_CH]) {
    T* ob = out + p0 + (int64_t)c * WAVE_CH * 64;
#pragma unroll
    for (int u = 0; u < WAVE_CH; ++u) {
      const T upv = lane_shr1(xv[u], yp);
      T acc = (T)0;
      if (UP_FIRST) {
        acc += op[u].cb * upv;
        acc += op[u].cl * yp;
      } else {
        acc += op[u].cl * yp;
        acc += op[u].cb * upv;
      }
      T y = op[u].b - acc;
      if (DIAG) y *= op[u].d;
      if (u > 0) st_agent(ob + (u - 1) * 64, yp);
      yp = y;
    }
    st_agent(ob + (WAVE_CH - 1) * 64, yp);
    lds_release();
    if (l == 0) __hip_atomic_store(&consumed, (c + 1) * WAVE_CH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  take(0, flag_of(0), opA, xA);
  int fnext = flag_of(1);
  for (int c = 0; c < nchunks; c += 2) {
    take(c + 1, fnext, opB, xB);
    fnext = flag_of(c + 2);
    run(c, opA, xA);
    if (c + 2 < nchunks) take(c + 2, fnext, opA, xA);
    fnext = flag_of(c + 3);
    run(c + 1, opB, xB);
  }
}

// ------------------------------------------------------------- 3D grids
// Factors with the structure of a 3D grid of nx x ny x nz cells: row
// k = (z * ny + y) * nx + x of a lower factor depends at most on k - 1 (same
// grid line), k - nx (same plane) and k - nx * ny; ILU(0) of a seven-point
// operator in natural order has exactly this structure.  A wave owns a tile
// of 8 x 8 grid lines, lane l = 8 zz + yy holding the line y = 8 ty + yy,
// z = 8 tz + zz, and walks x with a skew of yy + zz: at step s lane l treats
// x = s - yy - zz.  All three dependencies are then results of the previous
// step: x - 1 in the lane's own register, y - 1 in lane l - 1 (DPP shift),
// z - 1 in lane l - 8 (a lane permute).  Lanes on the tile's low-y face
// (yy = 0) take y - 1 from the tile before it in y (its lanes yy = 7, seven
// steps later in its walk), lanes on the low-z face from the tile before it
// in z, through memory (value-as-flag); a poller wave streams both faces into
// LDS rings.  Tiles are numbered w = tz * TY + ty, so both neighbours of a
// tile have lower indices, and a tile runs seven steps plus one
// publish-and-poll hop behind each of them: the longest chain is
// TY + TZ - 2 hops, against nx + ny + nz - 2 dependency levels for the
// general sweep.  Positions p = (w * S + s) * 64 + l with S = nx + 14
// rounded up to whole pairs of chunks; as for the 2D grid, out-of-grid
// positions hold zero coefficients and right-hand side, and the upper layout
// is the lower one read backwards (lanes, steps and tiles all reverse, which
// maps the reversed grid's tiles onto the same pattern).
constexpr int W3_CH = 4;
constexpr int W3_D = 2;
constexpr int W3_SLOTS = 10;
constexpr int W3_RING = W3_CH * W3_SLOTS;
constexpr int W3_PRODUCERS = 4;
constexpr int W3_XRING = 128;
constexpr int W3_THREADS = 64 * (2 + W3_PRODUCERS);
static_assert(W3_XRING % 8 == 0 && W3_XRING % W3_CH == 0, "ring rows must not wrap within a poll or a chunk");

// coefficients of one position of a 3D layout: z - 1, y - 1, x - 1
// neighbours (z + 1, y + 1, x + 1 for upper factors) and the reciprocal
// diagonal (unused by factors without one)
template <class T>
struct alignas(4 * sizeof(T)) Quad {
  T cz, cy, cx, d;
};
template <class T>
struct alignas(4 * sizeof(T)) WaveOp3 {
  T cz, cy, cx, b;
};

// lane l receives lane l - 8's value (lanes 0 .. 7 receive lanes 56 .. 63's,
// which the caller replaces); `addr` = ((l - 8) & 63) * 4
__device__ __forceinline__ int lane_up8(int addr, int v) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ __forceinline__ float lane_up8(int addr, float v) {
  return __builtin_bit_cast(float, lane_up8(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_up8(int addr, double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)lane_up8(addr, (int)(uint32_t)b);
  const uint32_t hi = (uint32_t)lane_up8(addr, (int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One workgroup per tile: wave 0 computes, waves 1 .. W3_PRODUCERS stream
// the operands into an LDS ring as in the 2D kernel, the last wave polls the
// two neighbouring tiles' faces.  LOWER: terms in the order z, y, x (the
// ascending column order of a lower factor), else x, y, z.  nb columns as in
// the 2D kernel: workgroup w * nb + r runs tile w of column r.
template <class T, bool DIAG, bool LOWER, bool REV>
__global__ __launch_bounds__(W3_THREADS) void k_wave3(int S, int TY, int64_t total, const Quad<T>* __restrict__ coef,
                                                      const T* __restrict__ rhs, T* out, int* abort_flag,
                                                      uint64_t limit, int nb) {
  __shared__ WaveOp3<T> r_op[W3_RING][64];
  __shared__ T r_d[DIAG ? W3_RING : 1][64];
  __shared__ T r_by[W3_XRING][8];  // face y - 1 of steps s (index zz)
  __shared__ T r_bz[W3_XRING][8];  // face z - 1 (index yy)
  __shared__ int ready[W3_SLOTS];
  __shared__ int xready;
  __shared__ int consumed;
  const int w = blockIdx.x / nb, l = threadIdx.x & 63, role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  {
    const int col = blockIdx.x - w * nb;
    rhs += (int64_t)col * total;
    out += (int64_t)col * total;
  }
  const int ty = w % TY, tz = w / TY;
  const int64_t p0 = (int64_t)w * S * 64 + l;
  const int nchunks = S / W3_CH;
  if (threadIdx.x < W3_SLOTS) ready[threadIdx.x] = 0;
  if (threadIdx.x == 0) { consumed = 0; xready = 0; }
  // the face rings start at zero: tiles on the grid's low faces read them
  // for every step against zero coefficients
  for (int i = threadIdx.x; i < W3_XRING * 8; i += W3_THREADS) {
    r_by[i >> 3][i & 7] = (T)0;
    r_bz[i >> 3][i & 7] = (T)0;
  }
  __syncthreads();

  // face values exist for steps s < xn (the neighbour's step s + 7); later
  // steps only meet zero coefficients
  const int xn = S - 7;
  const bool hy = ty > 0, hz = tz > 0;
  if (role == 1 + W3_PRODUCERS) {
    // ------------------------------------------- the neighbouring faces
    if (!hy && !hz) return;
    // lane l polls step next + l / 8: face y - 1 at zz = l % 8 (the y
    // neighbour's lane 8 zz + 7) and face z - 1 at yy = l % 8 (the z
    // neighbour's lane 56 + yy)
    const int j = l & 7, sl = l >> 3;
    const T* py = out + ((int64_t)(w - (hy ? 1 : 0)) * S + 7) * 64 + 8 * j + 7;
    const T* pz = out + ((int64_t)(w - (hz ? TY : 0)) * S + 7) * 64 + 56 + j;
    int next = 0;
    const uint64_t t0 = wall_clock64();
    unsigned it = 0;
#pragma clang loop unroll(disable)
    while (next < xn) {
      if (!wait_lds_at_least<4>(&consumed, next + 8 - W3_XRING, abort_flag, limit)) return;
      const int s = next + sl;
      T vy = (T)0, vz = (T)0;
      if (s < xn) {
        if (hy) vy = ld_agent(py + (int64_t)s * 64);
        if (hz) vz = ld_agent(pz + (int64_t)s * 64);
      }
      const uint64_t pend = __ballot(s < xn && (is_sentinel(vy) || is_sentinel(vz)));
      const int k = pend ? (int)(__builtin_ctzll(pend) >> 3) : 8;  // leading complete steps
      if (k > 0) {
        if (sl < k) {
          r_by[s % W3_XRING][j] = vy;
          r_bz[s % W3_XRING][j] = vz;
        }
        lds_release();
        next = std::min(next + k, xn);
        if (l == 0) __hip_atomic_store(&xready, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        __builtin_amdgcn_s_sleep(1);
        if ((++it & 63u) == 0) {
          if (ld_agent(abort_flag)) return;
          if (wall_clock64() - t0 > limit) {
            st_agent(abort_flag, 1);
            return;
          }
        }
      }
    }
    return;
  }

  if (role > 0) {
    // ---------------------------------------------------------- producer
    const int k = role - 1;
    Quad<T> rq[W3_D][W3_CH];
    T rb[W3_D][W3_CH];
    auto issue = [&](int c, int slot) {
#pragma unroll
      for (int u = 0; u < W3_CH; ++u) {
        const int64_t p = p0 + (int64_t)(c * W3_CH + u) * 64;
        rq[slot][u] = coef[p];
        rb[slot][u] = REV ? rhs[total - 1 - p] : rhs[p];
      }
    };
#pragma unroll
    for (int d = 0; d < W3_D; ++d) {
      const int c = k + d * W3_PRODUCERS;
      if (c < nchunks) issue(c, d);
    }
    for (int d0 = 0;; d0 += W3_D) {
#pragma unroll
      for (int dd = 0; dd < W3_D; ++dd) {
        const int c = k + (d0 + dd) * W3_PRODUCERS;
        if (c >= nchunks) return;
        if (!wait_lds_at_least<4>(&consumed, (c + 1 - W3_SLOTS) * W3_CH, abort_flag, limit)) return;
        const int rb0 = (c % W3_SLOTS) * W3_CH;
#pragma unroll
        for (int u = 0; u < W3_CH; ++u) {
          WaveOp3<T> op;
          op.cz = rq[dd][u].cz;
          op.cy = rq[dd][u].cy;
          op.cx = rq[dd][u].cx;
          op.b = is_sentinel(rb[dd][u]) ? (T)__builtin_nan("") : rb[dd][u];
          r_op[rb0 + u][l] = op;
          if (DIAG) r_d[rb0 + u][l] = rq[dd][u].d;
        }
        lds_release();
        if (l == 0) __hip_atomic_store(&ready[c % W3_SLOTS], c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int cn = c + W3_D * W3_PRODUCERS;
        if (cn < nchunks) issue(cn, dd);
      }
    }
  }

  // ------------------------------------------------------------ consumer
  // as in the 2D kernel: chunks two at a time, operand sets A and B
  const int yy = l & 7, zz = l >> 3;
  const int up8 = ((l - 8) & 63) << 2;
  const bool reads_faces = hy || hz;
  bool live = true;
  int seen_x = 0;
  WaveOp3<T> opA[W3_CH], opB[W3_CH];
  T dA[W3_CH], dB[W3_CH], yA[W3_CH], zA[W3_CH], yB[W3_CH], zB[W3_CH];
  auto flag_of = [&](int c) {
    return c < nchunks ? __hip_atomic_load(&ready[c % W3_SLOTS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                       : 0;
  };
  auto take = [&](int c, int seen, WaveOp3<T>(&op)[W3_CH], T(&dv)[W3_CH], T(&fy)[W3_CH], T(&fz)[W3_CH]) {
    const int slot = c % W3_SLOTS;
    if (live && seen != c + 1) live = wait_lds_equal(&ready[slot], c + 1, abort_flag, limit);
    const int s0 = c * W3_CH;
    if (reads_faces && s0 < xn) {
      const int need = std::min(s0 + W3_CH, xn);
      if (live && seen_x < need) {
        seen_x = __hip_atomic_load(&xready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (seen_x < need) {
          live = wait_lds_at_least<0, false>(&xready, need, abort_flag, limit);
          seen_x = need;
        }
      }
    }
    lds_acquire();
    const int r0 = slot * W3_CH, x0 = s0 % W3_XRING;
#pragma unroll
    for (int u = 0; u < W3_CH; ++u) {
      op[u] = r_op[r0 + u][l];
      if (DIAG) dv[u] = r_d[r0 + u][l];
      fy[u] = r_by[x0 + u][zz];
      fz[u] = r_bz[x0 + u][yy];
    }
  };
  T yp = (T)0;
  auto run = [&](int c, const WaveOp3<T>(&op)[W3_CH], const T(&dv)[W3_CH], const T(&fy)[W3_CH],
                 const T(&fz)[W3_CH]) {
    T* ob = out + p0 + (int64_t)c * W3_CH * 64;
#pragma unroll
    for (int u = 0; u < W3_CH; ++u) {
      const T sy = lane_shr1(fy[u], yp);
      const T sz = lane_up8(up8, yp);
      const T vy = yy == 0 ? fy[u] : sy;
      const T vz = zz == 0 ? fz[u] : sz;
      T acc = (T)0;
      if (LOWER) {
        acc += op[u].cz * vz;
        acc += op[u].cy * vy;
        acc += op[u].cx * yp;
      } else {
        acc += op[u].cx * yp;
        acc += op[u].cy * vy;
        acc += op[u].cz * vz;
      }
      T y = op[u].b - acc;
      if (DIAG) y *= dv[u];
      if (u > 0) st_agent(ob + (u - 1) * 64, yp);
      yp = y;
    }
    st_agent(ob + (W3_CH - 1) * 64, yp);
    lds_release();
    if (l == 0) __hip_atomic_store(&consumed, (c + 1) * W3_CH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  take(0, flag_of(0), opA, dA, yA, zA);
  int fnext = flag_of(1);
  for (int c = 0; c < nchunks; c += 2) {
    take(c + 1, fnext, opB, dB, yB, zB);
    fnext = flag_of(c + 2);
    run(c, opA, dA, yA, zA);
    if (c + 2 < nchunks) take(c + 2, fnext, opA, dA, yA, zA);
    fnext = flag_of(c + 3);
    run(c + 1, opB, dB, yB, zB);
  }
}

// positions of the lower layout -> cell (or -1 outside the grid)
struct WaveDims {
  int S, nx, ny, nz, TY;  // nz == 0: 2D grid
};
__device__ __forceinline__ int wave_cell(int64_t q, const WaveDims& g) {
  const int l = (int)(q & 63);
  const int64_t ws = q >> 6;
  const int w = (int)(ws / g.S), s = (int)(ws - (int64_t)w * g.S);
  if (g.nz == 0) {
    const int j = 64 * w + l, i = s - l;
    return (i >= 0 && i < g.nx && j < g.ny) ? j * g.nx + i : -1;
  }
  const int yy = l & 7, zz = l >> 3, ty = w % g.TY, tz = w / g.TY;
  const int x = s - yy - zz, y = 8 * ty + yy, z = 8 * tz + zz;
  return (x >= 0 && x < g.nx && y < g.ny && z < g.nz) ? (z * g.ny + y) * g.nx + x : -1;
}

// The gather takes the positions in tiles of 16 steps of one wave (or 3D
// tile): a lane's 16 cells of a tile are consecutive in x, at most two
// 128-byte lines of the cell-ordered vector, so a line is read by one or two
// workgroups (positions in plain grid-stride order spread a line's 16 values
// over four or five workgroups, usually on different XCDs and their L2s).
constexpr int WAVE_COPY_THREADS = 256;
constexpr int WAVE_COPY_TILE = 16 * 64;  // positions per tile

// column blockIdx.y: z + col * ldz (cell order) -> zs + col * total
template <class T, class TR>
__global__ __launch_bounds__(WAVE_COPY_THREADS) void k_wave_gather(int64_t total, WaveDims g,
                                                                   const TR* __restrict__ z, T* __restrict__ zs,
                                                                   size_t ldz) {
  z += blockIdx.y * ldz;
  zs += blockIdx.y * total;
  for (int64_t t0 = blockIdx.x * (int64_t)WAVE_COPY_TILE; t0 < total; t0 += (int64_t)gridDim.x * WAVE_COPY_TILE) {
    T v[WAVE_COPY_TILE / WAVE_COPY_THREADS];
#pragma unroll
    for (int k = 0; k < WAVE_COPY_TILE / WAVE_COPY_THREADS; ++k) {
      const int64_t p = t0 + k * WAVE_COPY_THREADS + threadIdx.x;
      const int c = p < total ? wave_cell(p, g) : -1;
      v[k] = c >= 0 ? (T)z[c] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < WAVE_COPY_TILE / WAVE_COPY_THREADS; ++k) {
      const int64_t p = t0 + k * WAVE_COPY_THREADS + threadIdx.x;
      if (p < total) zs[p] = v[k];
    }
  }
}

// out[cell] = ts[p] for the upper layout (cell of lower position total-1-p);
// ts and the lower sweep's output ys are reset to the sentinel for the next
// pair of sweeps.  Plain grid-stride order: its three streams of stores keep
// more workgroups busy than the tiled order (measured faster on 1024^2).
template <class T>
__global__ __launch_bounds__(WAVE_COPY_THREADS) void k_wave_scatter(int64_t total, WaveDims g, T* __restrict__ ts,
                                                                    T* __restrict__ ys, T* __restrict__ t,
                                                                    size_t ldt) {
  ts += blockIdx.y * total;
  ys += blockIdx.y * total;
  t += blockIdx.y * ldt;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = wave_cell(total - 1 - p, g);
    if (c >= 0) t[c] = ts[p];
    ts[p] = sentinel_of<T>(0);
    ys[total - 1 - p] = sentinel_of<T>(0);
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
                      T* ys, T* ts, T* t, int* abort_flag, hipStream_t s, int nb, size_t ldz, size_t ldt) {
  constexpr bool F32 = sizeof(T) == 4;
  using P2 = typename Pair<T>::type;
  const bool three = g.nz > 0;
  if (g.S % (2 * (three ? W3_CH : WAVE_CH)) != 0)
    fail(GMG_ERR_INVALID_ARG, "wavefront layout: steps not a multiple of two chunks");
  if (three && (g.TY < 1 || (int64_t)g.W * g.S * 64 != g.total || g.S < 8))
    fail(GMG_ERR_INVALID_ARG, "wavefront layout: inconsistent 3D tiling");
  if (nb < 1 || nb > 65535 || (int64_t)g.W * nb > INT32_MAX) fail(GMG_ERR_INVALID_ARG, "wavefront sweep: bad column count");
  const WaveDims dims{g.S, g.nx, g.ny, three ? g.nz : 0, three ? g.TY : 1};
  const unsigned gb = (unsigned)std::min<int64_t>(4096, (g.total + WAVE_COPY_TILE - 1) / WAVE_COPY_TILE);
  if (z_f64)
    hipLaunchKernelGGL((k_wave_gather<T, double>), dim3(gb, nb), dim3(WAVE_COPY_THREADS), 0, s, g.total, dims,
                       (const double*)z, zs, ldz);
  else
    hipLaunchKernelGGL((k_wave_gather<T, T>), dim3(gb, nb), dim3(WAVE_COPY_THREADS), 0, s, g.total, dims, (const T*)z,
                       zs, ldz);
  const uint64_t lim = wave_limit_ticks();
  const dim3 grid((unsigned)(g.W * nb));
  if (three) {
    // coefficient quads (z, y, x neighbours, reciprocal diagonal)
    auto co = [&](const WaveSweep& f) { return F32 ? (const Quad<T>*)f.coef32.p : (const Quad<T>*)f.coef.p; };
    const dim3 blk(W3_THREADS);
    if (lo.has_diag)
      hipLaunchKernelGGL((k_wave3<T, true, true, false>), grid, blk, 0, s, g.S, g.TY, g.total, co(lo), zs, ys,
                         abort_flag, lim, nb);
    else
      hipLaunchKernelGGL((k_wave3<T, false, true, false>), grid, blk, 0, s, g.S, g.TY, g.total, co(lo), zs, ys,
                         abort_flag, lim, nb);
    if (up.has_diag)
      hipLaunchKernelGGL((k_wave3<T, true, false, true>), grid, blk, 0, s, g.S, g.TY, g.total, co(up), ys, ts,
                         abort_flag, lim, nb);
    else
      hipLaunchKernelGGL((k_wave3<T, false, false, true>), grid, blk, 0, s, g.S, g.TY, g.total, co(up), ys, ts,
                         abort_flag, lim, nb);
  } else {
    auto co = [&](const WaveSweep& f) { return F32 ? (const P2*)f.coef32.p : (const P2*)f.coef.p; };
    auto di = [&](const WaveSweep& f) { return F32 ? (const T*)f.dinv32.p : (const T*)f.dinv.p; };
    // lower factor: neighbour below first; upper factor: left neighbour first,
    // right-hand side = the lower sweep's output read backwards
    const dim3 blk(WAVE_THREADS);
    if (lo.has_diag)
      hipLaunchKernelGGL((k_wave<T, true, true, false>), grid, blk, 0, s, g.S, g.nx, g.total, co(lo), di(lo), zs,
                         ys, abort_flag, lim, nb);
    else
      hipLaunchKernelGGL((k_wave<T, false, true, false>), grid, blk, 0, s, g.S, g.nx, g.total, co(lo), di(lo), zs,
                         ys, abort_flag, lim, nb);
    if (up.has_diag)
      hipLaunchKernelGGL((k_wave<T, true, false, true>), grid, blk, 0, s, g.S, g.nx, g.total, co(up), di(up), ys,
                         ts, abort_flag, lim, nb);
    else
      hipLaunchKernelGGL((k_wave<T, false, false, true>), grid, blk, 0, s, g.S, g.nx, g.total, co(up), di(up), ys,
                         ts, abort_flag, lim, nb);
  }
  const unsigned gs = (unsigned)std::min<int64_t>(4096, (g.total + WAVE_COPY_THREADS - 1) / WAVE_COPY_THREADS);
  hipLaunchKernelGGL((k_wave_scatter<T>), dim3(gs, nb), dim3(WAVE_COPY_THREADS), 0, s, g.total, dims, ts, ys, t, ldt);
  HIPCK(hipGetLastError());
}
template void launch_wave_pair<double>(const WaveGrid&, const WaveSweep&, const WaveSweep&, const void*, bool,
                                       double*, double*, double*, double*, int*, hipStream_t, int, size_t, size_t);
template void launch_wave_pair<float>(const WaveGrid&, const WaveSweep&, const WaveSweep&, const void*, bool,
                                      float*, float*, float*, float*, int*, hipStream_t, int, size_t, size_t);

}  // namespace gmg
