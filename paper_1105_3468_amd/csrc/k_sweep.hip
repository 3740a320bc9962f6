// Synchronisation-free triangular sweeps (smoother and coarse solve) and the
// level-synchronous ILU(0) factorisation.
//
// A sweep computes out[r] = (rhs[r] - sum_q dval[q] * out[dcol[q]]) * dinv[r]
// for every row of a triangular factor.  Rows are visited in a schedule of
// dependency levels, cut into wave-sized chunks that never mix two levels, so
// a wave never holds two rows where one depends on the other.  A chunk gives
// each of its rows G lanes (G a power of two chosen per level from the
// longest row, so that a lane reads at most one batch of entries); the lanes'
// partial sums meet in a shuffle reduction.  Waves take chunks from a global
// ticket counter in schedule order, so every row a wave waits for belongs to
// a chunk that an already-running wave holds: the sweep always makes
// progress.  A result is published with one relaxed agent-scope store
// and doubles as its own ready flag: consumers poll with relaxed agent-scope
// loads until the value differs from the NaN sentinel the buffer was reset to.
// Every wait is bounded by a wall-clock limit; a timeout raises a device flag
// that makes all other waits give up, so the grid always drains.
//
// Publishing through memory at agent scope costs about half a microsecond
// per hop (the XCDs' L2 caches are not coherent with each other), and that
// hop is the whole cost of a dependency level when levels hold only a few
// rows.  Such level ranges run on one workgroup instead (k_sweep_lds): the
// same chunks and the same arithmetic in the same order, tickets from an LDS
// counter, and the range's own results published in and polled from LDS (a
// copy also goes to global memory for later kernels).  Wide ranges keep the
// whole device for bandwidth.  Range boundaries are kernel boundaries, so a
// range reads the results of earlier ranges as final values.
#include <algorithm>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int SWEEP_BATCH = 8;
constexpr int SWEEP_WG_THREADS = 1024;  // the one workgroup of k_sweep_lds

template <class T>
__device__ __forceinline__ T not_sentinel(T v) {
  // a computed value equal to the sentinel's bits would never be seen as
  // ready; replace it by the canonical NaN (only reachable from NaN inputs)
  return is_sentinel(v) ? (T)__builtin_nan("") : v;
}

// Dependency values of the device-wide sweep: out[col], published at agent
// scope by any CU.
template <class T>
struct GlobalSrc {
  const T* out;
  static constexpr bool kSleep = true;  // polls cross the device: do not flood it
  __device__ void fetch(const int (&c)[SWEEP_BATCH], T (&v)[SWEEP_BATCH]) const {
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u) v[u] = ld_agent(out + c[u]);
  }
  __device__ unsigned pending(const int (&)[SWEEP_BATCH], const T (&v)[SWEEP_BATCH], unsigned need) const {
    unsigned p = 0;
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      if (is_sentinel(v[u])) p |= 1u << u;
    return p & need;
  }
  __device__ void refetch(const int (&c)[SWEEP_BATCH], T (&v)[SWEEP_BATCH], unsigned pend) const {
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      if (pend >> u & 1u) v[u] = ld_agent(out + c[u]);
  }
};

// Dependency values of the one-workgroup sweep: code >= 0 is the LDS slot of a
// row of this range; code < 0 is row -1 - code of an earlier range, final in
// global memory.  Both loads are issued for every entry (the unused one at a
// clamped address) and the result selected, so a batch is straight-line code
// with all its loads in flight together.
template <class T>
struct LdsSrc {
  T* xs;
  const T* out;
  static constexpr bool kSleep = false;  // LDS polls are cheap and local
  __device__ void fetch(const int (&c)[SWEEP_BATCH], T (&v)[SWEEP_BATCH]) const {
    T g[SWEEP_BATCH], l[SWEEP_BATCH];
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u) g[u] = out[c[u] < 0 ? -1 - c[u] : 0];
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      l[u] = __hip_atomic_load(xs + (c[u] >= 0 ? c[u] : 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u) v[u] = c[u] >= 0 ? l[u] : g[u];
  }
  __device__ unsigned pending(const int (&c)[SWEEP_BATCH], const T (&v)[SWEEP_BATCH], unsigned need) const {
    unsigned p = 0;
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      if (c[u] >= 0 && is_sentinel(v[u])) p |= 1u << u;
    return p & need;
  }
  __device__ void refetch(const int (&c)[SWEEP_BATCH], T (&v)[SWEEP_BATCH], unsigned pend) const {
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      if (pend >> u & 1u) v[u] = __hip_atomic_load(xs + c[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Dependency values that are final before the launch (rows of earlier
// levels, each level its own launch): plain loads, nothing to poll.
template <class T>
struct FinalSrc {
  const T* out;
  static constexpr bool kSleep = false;
  __device__ void fetch(const int (&c)[SWEEP_BATCH], T (&v)[SWEEP_BATCH]) const {
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u) v[u] = out[c[u]];
  }
  __device__ unsigned pending(const int (&)[SWEEP_BATCH], const T (&)[SWEEP_BATCH], unsigned) const { return 0u; }
  __device__ void refetch(const int (&)[SWEEP_BATCH], T (&)[SWEEP_BATCH], unsigned) const {}
};

// acc = sum of this lane's share of row e's entries: entries q0+sub,
// q0+sub+G, ... (q0 < q1), SWEEP_BATCH at a time.  Every batch loads its
// entries unconditionally (past the row's end at the row's last entry, not
// added) so all its loads are in flight together.  Values not yet published
// are polled as a group: every round re-issues all of them together, so a
// round costs one latency however many are pending.  Entries are added in
// ascending order in both sweeps, so they give bitwise identical sums.
template <class T, class Src>
__device__ __forceinline__ T lane_partial(const Src& src, const int* __restrict__ dref,
                                          const T* __restrict__ dval, int q0, int q1, int G, int* abort_flag,
                                          uint64_t limit) {
  T acc = (T)0;
  for (int q = q0; q < q1; q += G * SWEEP_BATCH) {
    int c[SWEEP_BATCH];
    T v[SWEEP_BATCH];
    T a[SWEEP_BATCH];
    unsigned need = 0;
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u) {
      const int qq = q + u * G < q1 ? q + u * G : q1 - 1;
      c[u] = dref[qq];
      a[u] = dval[qq];
      if (q + u * G < q1) need |= 1u << u;
    }
    src.fetch(c, v);
    unsigned pend = src.pending(c, v, need);
    if (pend) {
      const uint64_t t0 = wall_clock64();
      unsigned it = 0;
#pragma clang loop unroll(disable)
      while (pend) {
        if constexpr (Src::kSleep) __builtin_amdgcn_s_sleep(1);
        src.refetch(c, v, pend);
        pend = src.pending(c, v, pend);
        if (pend && (++it & 63u) == 0) {
          bool give_up = ld_agent(abort_flag) != 0;
          if (!give_up && wall_clock64() - t0 > limit) {
            st_agent(abort_flag, 1);
            give_up = true;
          }
          if (give_up) {
#pragma unroll
            for (int u = 0; u < SWEEP_BATCH; ++u)
              if (pend >> u & 1u) v[u] = (T)__builtin_nan("");
            pend = 0;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SWEEP_BATCH; ++u)
      if (need >> u & 1u) acc += a[u] * v[u];
  }
  return acc;
}

// The rows of one chunk: lanes grouped per row, partial sums reduced by
// shuffles, the row's owner lane stores.  The row's own operands (index,
// right-hand side, reciprocal diagonal) do not depend on other rows and are
// loaded before the dependencies, so only the reduction and the store follow
// the last dependency.  Returns, for the owner lane, the row's entry and value;
// the caller publishes the value and only then resets the right-hand side
// (stores count against the same wait counter as loads, so a store issued
// before the value is computed would be waited for on the critical path).
template <class T, class TR, bool DIAG, class Src>
__device__ __forceinline__ bool chunk_rows(const Src& src, const int* __restrict__ chunk, unsigned t,
                                           const int* __restrict__ rows, const int* __restrict__ dp,
                                           const int* __restrict__ dref, const T* __restrict__ dval,
                                           const T* __restrict__ dinv, const TR* rhs, int* abort_flag,
                                           uint64_t limit, int& e_out, int& r_out, T& y_out) {
  const int lane = threadIdx.x & 63;
  // chunk: first entry, number of rows, log2 of lanes per row
  const int c0 = chunk[3 * t], cr = chunk[3 * t + 1], lg = chunk[3 * t + 2];
  const int G = 1 << lg;
  const int slot = lane >> lg, sub = lane & (G - 1);
  const bool active = slot < cr;
  const int e = c0 + slot;
  int r = 0;
  T rh = (T)0, di = (T)1;
  if (active && sub == 0) {
    r = rows[e];
    rh = (T)rhs[r];
    if (DIAG) di = dinv[r];
  }
  T acc = (T)0;
  if (active) acc = lane_partial<T>(src, dref, dval, dp[e] + sub, dp[e + 1], G, abort_flag, limit);
  for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!(active && sub == 0)) return false;
  T y = rh - acc;
  if (DIAG) y *= di;
  e_out = e;
  r_out = r;
  y_out = not_sentinel(y);
  return true;
}

template <class T, class TR, bool DIAG>
__global__ __launch_bounds__(256) void k_sweep(const int* __restrict__ chunk, const int* __restrict__ rows,
                                               const int* __restrict__ dp, const int* __restrict__ dcol,
                                               const T* __restrict__ dval, const T* __restrict__ dinv,
                                               const TR* rhs, T* out, TR* reset_rhs, unsigned nchunks,
                                               unsigned* ticket, unsigned base, int* abort_flag, uint64_t limit) {
  const int lane = threadIdx.x & 63;
  const GlobalSrc<T> src{out};
  for (;;) {
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(ticket, 1u) - base;
    t = __shfl(t, 0, 64);
    if (t >= nchunks) break;
    int e, r;
    T y;
    if (chunk_rows<T, TR, DIAG>(src, chunk, t, rows, dp, dcol, dval, dinv, rhs, abort_flag, limit, e, r, y)) {
      st_agent(out + r, y);
      // rhs and reset_rhs may be the same buffer: the row read it already
      if (reset_rhs) reset_rhs[r] = sentinel_of<TR>(0);
    }
  }
}

// The chunks of one dependency level, a wave per chunk: every dependency
// belongs to an earlier level, complete when this launch starts, so the
// values are read as they are.  Used for factors with a few wide levels (the
// colour classes of a multicolour ordering), where one launch per level costs
// less than the device-wide sweep's publishing and polling.
template <class T, class TR, bool DIAG>
__global__ __launch_bounds__(256) void k_sweep_level(const int* __restrict__ chunk, const int* __restrict__ rows,
                                                     const int* __restrict__ dp, const int* __restrict__ dcol,
                                                     const T* __restrict__ dval, const T* __restrict__ dinv,
                                                     const TR* rhs, T* out, TR* reset_rhs, unsigned nchunks) {
  const unsigned t = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (t >= nchunks) return;
  const FinalSrc<T> src{out};
  int e, r;
  T y;
  if (chunk_rows<T, TR, DIAG>(src, chunk, t, rows, dp, dcol, dval, dinv, rhs, nullptr, 0, e, r, y)) {
    out[r] = y;
    if (reset_rhs) reset_rhs[r] = sentinel_of<TR>(0);
  }
}

// One workgroup over the chunks of a level range whose rows are entries
// [e0, e0 + m); their results live in LDS slots e - e0 (dynamic LDS of m
// values, reset to the sentinel at start).  dslot holds the LDS slot or the
// -1 - row code of every dependency entry of the range.
template <class T, class TR, bool DIAG>
__global__ __launch_bounds__(SWEEP_WG_THREADS) void k_sweep_lds(
    const int* __restrict__ chunk, const int* __restrict__ rows, const int* __restrict__ dp,
    const int* __restrict__ dslot, const T* __restrict__ dval, const T* __restrict__ dinv, const TR* rhs, T* out,
    TR* reset_rhs, unsigned nchunks, int e0, int m, int* abort_flag, uint64_t limit) {
  extern __shared__ __align__(16) unsigned char sweep_smem[];
  T* xs = reinterpret_cast<T*>(sweep_smem);
  __shared__ unsigned ticket;
  for (int i = threadIdx.x; i < m; i += SWEEP_WG_THREADS) xs[i] = sentinel_of<T>(0);
  if (threadIdx.x == 0) ticket = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const LdsSrc<T> src{xs, out};
  for (;;) {
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(&ticket, 1u);
    t = __shfl(t, 0, 64);
    if (t >= nchunks) break;
    int e, r;
    T y;
    if (chunk_rows<T, TR, DIAG>(src, chunk, t, rows, dp, dslot, dval, dinv, rhs, abort_flag, limit, e, r, y)) {
      __hip_atomic_store(xs + (e - e0), y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      out[r] = y;
      if (reset_rhs) reset_rhs[r] = sentinel_of<TR>(0);
    }
  }
}

static uint64_t wall_limit_ticks() {
  static uint64_t ticks = 0;
  if (!ticks) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
      (void)hipGetLastError();
      khz = 100000;  // 100 MHz
    }
    ticks = (uint64_t)khz * 1000ull * 4ull;  // 4 seconds
  }
  return ticks;
}

template <class T>
void launch_sweep_levels(Sweep& sw, const T* dval, const T* dinv, const void* rhs, bool rhs_is_f64, T* out,
                         T* reset_rhs, hipStream_t s) {
  if (sw.nchunks == 0) return;
  if ((int)sw.lvl_c0.size() != sw.levels + 1) fail(GMG_ERR_INVALID_ARG, "level sweep: no level table");
  for (int l = 0; l < sw.levels; ++l) {
    const int c0 = sw.lvl_c0[l];
    const unsigned nchunks = (unsigned)(sw.lvl_c0[l + 1] - c0);
    if (nchunks == 0) continue;
    const int* ch = sw.chunk.p + 3 * (size_t)c0;
    const unsigned blocks = (nchunks + 3) / 4;
#define GMG_SWV(TR_, DG_, RHS_, RESET_)                                                                       \
  hipLaunchKernelGGL((k_sweep_level<T, TR_, DG_>), dim3(blocks), dim3(256), 0, s, ch, sw.rows.p, sw.dp.p,    \
                     sw.dcol.p, dval, dinv, (const TR_*)RHS_, out, RESET_, nchunks)
    if (rhs_is_f64 && sizeof(T) == 4) {
      if (sw.has_diag) GMG_SWV(double, true, rhs, (double*)nullptr);
      else GMG_SWV(double, false, rhs, (double*)nullptr);
    } else {
      if (sw.has_diag) GMG_SWV(T, true, rhs, reset_rhs);
      else GMG_SWV(T, false, rhs, reset_rhs);
    }
#undef GMG_SWV
    HIPCK(hipGetLastError());
  }
}
template void launch_sweep_levels<double>(Sweep&, const double*, const double*, const void*, bool, double*, double*,
                                          hipStream_t);
template void launch_sweep_levels<float>(Sweep&, const float*, const float*, const void*, bool, float*, float*,
                                         hipStream_t);

template <class T>
void launch_sweep(Sweep& sw, const T* dval, const T* dinv, const void* rhs, bool rhs_is_f64, T* out,
                  T* reset_rhs, int waves, bool whole, int* abort_flag, hipStream_t s) {
  if (sw.nchunks == 0) return;
  const uint64_t lim = wall_limit_ticks();
  // whole: every level device-wide in one launch; else the level ranges
  // chosen at setup
  const int nseg = whole ? 1 : (int)sw.seg_c0.size();
  for (int g = 0; g < nseg; ++g) {
    const int c0 = whole ? 0 : sw.seg_c0[g];
    const unsigned nchunks = (unsigned)((whole ? sw.nchunks : sw.seg_c1[g]) - c0);
    const bool wg = !whole && sw.seg_wg[g] != 0;
    const int* ch = sw.chunk.p + 3 * (size_t)c0;
    if (nchunks == 0) continue;
    if (wg) {
      const int e0 = sw.seg_e0[g], m = sw.seg_e1[g] - e0;
      const size_t lds = (size_t)m * sizeof(T);
#define GMG_SWL(TR_, DG_, RHS_, RESET_)                                                                            \
  do {                                                                                                            \
    static bool attr = false;                                                                                     \
    if (!attr) {                                                                                                  \
      HIPCK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_lds<T, TR_, DG_>),                         \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kSweepLdsRows * sizeof(double)))); \
      attr = true;                                                                                                \
    }                                                                                                             \
    hipLaunchKernelGGL((k_sweep_lds<T, TR_, DG_>), dim3(1), dim3(SWEEP_WG_THREADS), lds, s, ch, sw.rows.p,        \
                       sw.dp.p, sw.dslot.p, dval, dinv, (const TR_*)RHS_, out, RESET_, nchunks, e0, m, abort_flag, lim); \
  } while (0)
      if (rhs_is_f64 && sizeof(T) == 4) {
        if (sw.has_diag) GMG_SWL(double, true, rhs, (double*)nullptr);
        else GMG_SWL(double, false, rhs, (double*)nullptr);
      } else {
        if (sw.has_diag) GMG_SWL(T, true, rhs, reset_rhs);
        else GMG_SWL(T, false, rhs, reset_rhs);
      }
#undef GMG_SWL
      HIPCK(hipGetLastError());
      continue;
    }
    unsigned w = waves > 0 ? (unsigned)waves : 2048u;
    if (w > nchunks) w = nchunks;
    const unsigned blocks = (w + 3) / 4;
    const unsigned used = blocks * 4;  // every wave takes exactly one ticket that ends it
#define GMG_SW(TR_, DG_, RHS_, RESET_)                                                                        \
  hipLaunchKernelGGL((k_sweep<T, TR_, DG_>), dim3(blocks), dim3(256), 0, s, ch, sw.rows.p, sw.dp.p, sw.dcol.p, \
                     dval, dinv, (const TR_*)RHS_, out, RESET_, nchunks, sw.ticket.p, sw.ticket_base, abort_flag, lim)
    if (rhs_is_f64 && sizeof(T) == 4) {
      // FP32 sweep with an FP64 right-hand side (first sweep of the FP32 cycle)
      if (sw.has_diag) GMG_SW(double, true, rhs, (double*)nullptr);
      else GMG_SW(double, false, rhs, (double*)nullptr);
    } else {
      if (sw.has_diag) GMG_SW(T, true, rhs, reset_rhs);
      else GMG_SW(T, false, rhs, reset_rhs);
    }
#undef GMG_SW
    HIPCK(hipGetLastError());
    sw.ticket_base += nchunks + used;
  }
}
template void launch_sweep<double>(Sweep&, const double*, const double*, const void*, bool, double*, double*,
                                   int, bool, int*, hipStream_t);
template void launch_sweep<float>(Sweep&, const float*, const float*, const void*, bool, float*, float*, int,
                                  bool, int*, hipStream_t);


// ------------------------------------------------------- single-CU sweep
// For factors whose dependency levels are narrow (at most CU_THREADS rows)
// and whose rows depend only on the previous two levels, one workgroup walks
// all levels itself: thread t computes the row at position t of each level,
// the values of the last three levels stay in an LDS ring (a level writes the
// slot its successor does not read), and one
// workgroup barrier separates consecutive levels.  A level then costs a
// barrier and a few LDS reads instead of a global-memory hop between compute
// units.  Operands are laid out per level in schedule order (rhs gathered
// before, result scattered after, by the two parallel kernels below), so
// every thread prefetches its operands PF levels ahead.
constexpr int CU_THREADS = 1024;
constexpr int CU_RING = 3;
constexpr int CU_MAX_LEVELS = 16400;

// The operands of entry e (W slots, W values) with as few vector loads as the
// width allows.
template <class T, int W>
__device__ __forceinline__ void load_ops(const int* __restrict__ wslot, const T* __restrict__ wval, int e,
                                         int (&ps)[W], T (&pv)[W]) {
  if constexpr (W == 2) {
    const int2 sl = *reinterpret_cast<const int2*>(wslot + (size_t)e * 2);
    ps[0] = sl.x;
    ps[1] = sl.y;
    if constexpr (sizeof(T) == 8) {
      const double2 v = *reinterpret_cast<const double2*>(wval + (size_t)e * 2);
      pv[0] = v.x;
      pv[1] = v.y;
    } else {
      const float2 v = *reinterpret_cast<const float2*>(wval + (size_t)e * 2);
      pv[0] = v.x;
      pv[1] = v.y;
    }
  } else if constexpr (W == 4) {
    const int4 sl = *reinterpret_cast<const int4*>(wslot + (size_t)e * 4);
    ps[0] = sl.x;
    ps[1] = sl.y;
    ps[2] = sl.z;
    ps[3] = sl.w;
    if constexpr (sizeof(T) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(wval + (size_t)e * 4);
      const double2 b = *reinterpret_cast<const double2*>(wval + (size_t)e * 4 + 2);
      pv[0] = a.x;
      pv[1] = a.y;
      pv[2] = b.x;
      pv[3] = b.y;
    } else {
      const float4 v = *reinterpret_cast<const float4*>(wval + (size_t)e * 4);
      pv[0] = v.x;
      pv[1] = v.y;
      pv[2] = v.z;
      pv[3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      ps[k] = wslot[(size_t)e * W + k];
      pv[k] = wval[(size_t)e * W + k];
    }
  }
}

template <class T, int W, int PF, bool DIAG>
__global__ __launch_bounds__(CU_THREADS) void k_cu_sweep(int levels, int dummy, const int* __restrict__ lptr,
                                                         const int* __restrict__ wslot, const T* __restrict__ wval,
                                                         const T* __restrict__ dinv_e, const T* __restrict__ rhs_s,
                                                         T* __restrict__ out_s) {
  // ring slots: 3 levels x CU_THREADS, then a zero (padding operand) and a
  // sink (results of idle threads)
  __shared__ T ring[CU_RING * CU_THREADS + 2];
  __shared__ int lp[CU_MAX_LEVELS + 1];
  const int t = threadIdx.x;
  const int padded = (levels + PF - 1) / PF * PF;
  if (t == 0) ring[CU_RING * CU_THREADS] = (T)0;
  // level bounds in LDS (levels past the end are empty), so prefetches never
  // wait on a global load
  for (int l = t; l <= padded + PF; l += CU_THREADS) lp[l] = lptr[min(l, levels)];
  __syncthreads();
  // register pipeline: operands of levels l .. l+PF-1.  Every load is issued
  // unconditionally (idle slots read the dummy entry), so the compiler can
  // count outstanding loads exactly and waits only for the oldest level.
  int pe[PF];
  T pr[PF], pd[PF], pv[PF][W];
  int ps[PF][W];
  const int wave0 = t & ~63;
  auto fetch = [&](int l, int u) {
    const int s0 = lp[l], s1 = lp[l + 1];
    const int e = s0 + t < s1 ? s0 + t : dummy;
    pe[u] = e;
    // waves with no row in this level load nothing (a wave-uniform branch)
    if (s0 + wave0 < s1) {
      pr[u] = rhs_s[e];
      pd[u] = DIAG ? dinv_e[e] : (T)1;
      load_ops<T, W>(wslot, wval, e, ps[u], pv[u]);
    } else {
      pr[u] = (T)0;
      pd[u] = (T)0;
#pragma unroll
      for (int k = 0; k < W; ++k) { ps[u][k] = CU_RING * CU_THREADS; pv[u][k] = (T)0; }
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) fetch(u, u);
  for (int l0 = 0; l0 < padded; l0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int l = l0 + u;
      T acc = (T)0;
#pragma unroll
      for (int k = 0; k < W; ++k) acc += pv[u][k] * ring[ps[u][k]];
      T y = pr[u] - acc;
      if (DIAG) y *= pd[u];
      const int slot = pe[u] != dummy ? (l % CU_RING) * CU_THREADS + t : CU_RING * CU_THREADS + 1;
      ring[slot] = y;
      out_s[pe[u]] = y;
      fetch(l + PF, u);
      // order the LDS ring only: a full __syncthreads() would also wait for
      // the prefetched global loads and serialise every level on memory
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
  }
}

template <class T, class TR>
__global__ void k_cu_gather(int n, const int* __restrict__ rows, const TR* rhs, TR* reset_rhs, T* __restrict__ rhs_s) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int r = rows[e];
    rhs_s[e] = (T)rhs[r];
    if (reset_rhs) reset_rhs[r] = sentinel_of<TR>(0);
  }
}

template <class T>
__global__ void k_cu_scatter(int n, const int* __restrict__ rows, const T* __restrict__ out_s, T* out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) out[rows[e]] = out_s[e];
}

template <class T>
void launch_cu_sweep(CuSweep& cs, const T* wval, const T* dinv_e, const void* rhs, bool rhs_is_f64, T* out,
                     T* reset_rhs, T* rhs_s, T* out_s, hipStream_t s) {
  const int n = cs.n;
  if (n <= 0) return;
  unsigned g = (unsigned)std::min<int64_t>(8192, (n + 255) / 256);
  if (rhs_is_f64 && sizeof(T) == 4)
    hipLaunchKernelGGL((k_cu_gather<T, double>), dim3(g), dim3(256), 0, s, n, cs.rows.p, (const double*)rhs,
                       (double*)nullptr, rhs_s);
  else
    hipLaunchKernelGGL((k_cu_gather<T, T>), dim3(g), dim3(256), 0, s, n, cs.rows.p, (const T*)rhs, reset_rhs,
                       rhs_s);
#define GMG_CU(W_, PF_)                                                                                       \
  do {                                                                                                        \
    if (cs.has_diag)                                                                                          \
      hipLaunchKernelGGL((k_cu_sweep<T, W_, PF_, true>), dim3(1), dim3(CU_THREADS), 0, s, cs.levels, n,       \
                         cs.lptr.p, cs.wslot.p, wval, dinv_e, rhs_s, out_s);                                  \
    else                                                                                                      \
      hipLaunchKernelGGL((k_cu_sweep<T, W_, PF_, false>), dim3(1), dim3(CU_THREADS), 0, s, cs.levels, n,      \
                         cs.lptr.p, cs.wslot.p, wval, dinv_e, rhs_s, out_s);                                  \
  } while (0)
  // prefetch depth within the 128-register budget of 1024-thread workgroups
  switch (cs.width) {
    case 1: GMG_CU(1, 8); break;
    case 2: GMG_CU(2, 8); break;
    case 3: GMG_CU(3, 4); break;
    default: GMG_CU(4, 4); break;
  }
#undef GMG_CU
  hipLaunchKernelGGL((k_cu_scatter<T>), dim3(g), dim3(256), 0, s, n, cs.rows.p, out_s, out);
  HIPCK(hipGetLastError());
}
template void launch_cu_sweep<double>(CuSweep&, const double*, const double*, const void*, bool, double*, double*,
                                      double*, double*, hipStream_t);
template void launch_cu_sweep<float>(CuSweep&, const float*, const float*, const void*, bool, float*, float*,
                                     float*, float*, hipStream_t);

// ------------------------------------------------------------------ ILU(0)
// One launch per dependency level of L0: every row of the level runs the IKJ
// elimination on its own entries, reading only rows of earlier levels, which
// are final.  Operation order and rounding follow the plain definition (no
// FMA contraction), so the factors are reproducible bit for bit.
#pragma clang fp contract(off)
__global__ void k_ilu0_level(const int* __restrict__ rows, int count, const int* __restrict__ rp,
                             const int* __restrict__ ci, const int* __restrict__ dpos, double* a, int* bad) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = rows[t];
  if (i < 0) return;
  const int p0 = rp[i], p1 = rp[i + 1], di = dpos[i];
  for (int p = p0; p < di; ++p) {
    const int k = ci[p];
    const double lik = a[p] / a[dpos[k]];
    a[p] = lik;
    int lo = p + 1;  // entries of row i with column > k start after p
    for (int r = dpos[k] + 1; r < rp[k + 1]; ++r) {
      const int j = ci[r];
      // row i columns ascending and U row k ascending: merge walk
      while (lo < p1 && ci[lo] < j) ++lo;
      if (lo >= p1) break;
      if (ci[lo] == j) a[lo] = a[lo] - lik * a[r];
    }
  }
  const double d = a[di];
  if (d == 0.0) atomicOr(bad, 1);
  else if (!isfinite(d)) atomicOr(bad, 2);
}
#pragma clang fp contract(on)

// ILU(0) of a matrix with the 2D-grid structure of the wavefront sweeps (row
// k = iy * nx + ix couples only to k -/+ 1 within its grid row and k -/+ nx;
// nx >= 3): the elimination of row i only updates its diagonal,
//   l1 = a(i, i-nx) / u(i-nx, i-nx);  d = a_ii - l1 * a(i-nx, i);
//   l2 = a(i, i-1)  / u(i-1, i-1);    d = d - l2 * a(i-1, i),
// (the terms of absent neighbours left out) in the order of the IKJ
// definition, so the result is the level-scheduled kernel's bit for bit.  A
// pivot depends on the previous anti-diagonal only: one workgroup walks the
// nx + ny - 1 anti-diagonals, thread y owning grid row y (and y + 1024, ...),
// with the previous diagonal's pivots in LDS and the next diagonal's
// operands loaded before the barrier.
// op[5 * i ..]: a_ii, a(i, i-nx), a(i-nx, i), a(i, i-1), a(i-1, i) (0 when
// absent); pos[2 * i ..]: positions of a(i, i-nx) and a(i, i-1) (or -1).
constexpr int ILUG_THREADS = 1024;
constexpr int ILUG_ROWS = 4;     // grid rows per thread at most (ny <= 4096)

__global__ void k_ilu0_grid_ops(int n, int nx, const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ dpos, const double* __restrict__ a, double* __restrict__ op,
                                int* __restrict__ pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = dpos[i];
  double o[5] = {a[d], 0.0, 0.0, 0.0, 0.0};
  int pd = -1, pl = -1;
  for (int p = rp[i]; p < d; ++p) {
    if (ci[p] == i - nx) pd = p;
    if (ci[p] == i - 1) pl = p;
  }
  if (pd >= 0) {
    o[1] = a[pd];
    const int k = i - nx;
    for (int p = dpos[k] + 1; p < rp[k + 1]; ++p)
      if (ci[p] == i) o[2] = a[p];
  }
  if (pl >= 0) {
    o[3] = a[pl];
    const int k = i - 1;
    for (int p = dpos[k] + 1; p < rp[k + 1]; ++p)
      if (ci[p] == i) o[4] = a[p];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) op[5 * (size_t)i + q] = o[q];
  pos[2 * (size_t)i] = pd;
  pos[2 * (size_t)i + 1] = pl;
}

#pragma clang fp contract(off)
__global__ __launch_bounds__(ILUG_THREADS) void k_ilu0_grid(int nx, int ny, const double* __restrict__ op,
                                                            const int* __restrict__ pos, const int* __restrict__ dpos,
                                                            double* __restrict__ a, int* bad) {
  extern __shared__ double piv[];   // two diagonals of pivots, indexed by grid row
  double* cur = piv;
  double* prv = piv + ny;
  const int steps = nx + ny - 1;
  double o[ILUG_ROWS][5];
  auto load = [&](int t) {
#pragma unroll
    for (int r = 0; r < ILUG_ROWS; ++r) {
      const int y = threadIdx.x + r * ILUG_THREADS, x = t - y;
      if (y < ny && x >= 0 && x < nx) {
        const size_t i = (size_t)y * nx + x;
#pragma unroll
        for (int q = 0; q < 5; ++q) o[r][q] = op[5 * i + q];
      }
    }
  };
  load(0);
  int flags = 0;
  for (int t = 0; t < steps; ++t) {
    double d[ILUG_ROWS];
#pragma unroll
    for (int r = 0; r < ILUG_ROWS; ++r) {
      const int y = threadIdx.x + r * ILUG_THREADS, x = t - y;
      d[r] = 0.0;
      if (y < ny && x >= 0 && x < nx) {
        const size_t i = (size_t)y * nx + x;
        double v = o[r][0];
        const int pd = pos[2 * i], pl = pos[2 * i + 1];
        if (pd >= 0) {
          const double l1 = o[r][1] / prv[y - 1];    // pivot of (x, y - 1), diagonal t - 1
          a[pd] = l1;
          v = v - l1 * o[r][2];
        }
        if (pl >= 0) {
          const double l2 = o[r][3] / prv[y];        // pivot of (x - 1, y), diagonal t - 1
          a[pl] = l2;
          v = v - l2 * o[r][4];
        }
        a[dpos[i]] = v;
        d[r] = v;
        if (v == 0.0) flags |= 1;
        else if (!isfinite(v)) flags |= 2;
      }
    }
    if (t + 1 < steps) load(t + 1);
#pragma unroll
    for (int r = 0; r < ILUG_ROWS; ++r) {
      const int y = threadIdx.x + r * ILUG_THREADS;
      if (y < ny) cur[y] = d[r];
    }
    __syncthreads();
    double* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  if (flags) atomicOr(bad, flags);
}
#pragma clang fp contract(on)

bool ilu0_grid_fits(int nx, int ny) { return nx >= 3 && ny >= 1 && ny <= ILUG_THREADS * ILUG_ROWS; }

void launch_ilu0_grid(int n, int nx, const int* rp, const int* ci, const int* dpos, double* a, int* bad,
                      hipStream_t s) {
  const int ny = n / nx;
  if (!ilu0_grid_fits(nx, ny) || (int64_t)nx * ny != n) fail(GMG_ERR_INVALID_ARG, "grid ILU(0): unsupported shape");
  DBuf<double> op;
  DBuf<int> pos;
  op.alloc((size_t)5 * n);
  pos.alloc((size_t)2 * n);
  hipLaunchKernelGGL(k_ilu0_grid_ops, dim3((n + 255) / 256), dim3(256), 0, s, n, nx, rp, ci, dpos, a, op.p, pos.p);
  const size_t lds = (size_t)2 * ny * sizeof(double);
  hipLaunchKernelGGL(k_ilu0_grid, dim3(1), dim3(ILUG_THREADS), lds, s, nx, ny, op.p, pos.p, dpos, a, bad);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(s));   // before op and pos are freed
}

void launch_ilu0_level(const int* rows, int count, const int* rp, const int* ci, const int* dpos, double* a,
                       int* bad, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ilu0_level, dim3((count + 255) / 256), dim3(256), 0, s, rows, count, rp, ci, dpos, a,
                     bad);
  HIPCK(hipGetLastError());
}

// ------------------------------------------------- Jacobi sweep on a factor
// yout[i] = (b[i] - sum_{j != i} F_ij yin[j]) * (dinv ? dinv[i] : 1)
__global__ void k_jacobi(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                         const double* __restrict__ v, const double* __restrict__ dinv,
                         const double* __restrict__ b, const double* __restrict__ yin,
                         double* __restrict__ yout) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = b[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    if (j != i) s -= v[p] * yin[j];
  }
  yout[i] = dinv ? s * dinv[i] : s;
}

void launch_jacobi(int n, const int* rp, const int* ci, const double* v, const double* dinv, const double* b,
                   const double* yin, double* yout, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_jacobi, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, v, dinv, b, yin, yout);
  HIPCK(hipGetLastError());
}

}  // namespace gmg
