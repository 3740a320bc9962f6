// Triangular solves over the nested-dissection tree (coarse ILUT factors).
//
// With the coarse unknowns numbered by nested dissection, an elimination only
// creates entries between a row and the rows of its own tree node or of the
// node's descendants (strictly lower part) or ancestors (strictly upper
// part).  So a lower solve can run bottom-up over the tree and an upper solve
// top-down, one node at a time along a root-leaf path, every node solving
// with its own diagonal block after subtracting the terms of rows outside it,
// which are final by then.  The diagonal blocks of separators are nearly dense
// after fill; they are stored dense (column-major, zeros where the factor
// has no entry) and solved in panels of 64 rows: one wave walks the panel's
// columns, broadcasting each finished value with readlane (zeros of the
// other triangle leave finished rows unchanged), and the workgroup then
// applies the panel to the node's remaining rows.  A level sweep would pay
// one dependency hop per row of a separator chain instead.
//
// One launch runs a whole solve as a list of tasks in tree order (lower:
// heights ascending; upper: descending).  For a node with terms outside it,
// helper tasks first compute rhs - (those terms) for slices of its rows,
// polling the published results of other nodes (value-as-flag, as in the
// sweeps), and publish them to a staging vector that doubles as its own
// ready flag; the node's own task polls them, solves, and publishes its rows.
// Every task waits only on earlier tasks and workgroups start in order, so
// the solve always makes progress; every wait is bounded.
#include <algorithm>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int TREE_THREADS = 256;
constexpr int TREE_BATCH = 8;

template <class T>
__device__ __forceinline__ T tree_poll(const T* p, int* abort_flag, uint64_t limit) {
  T v = ld_agent(p);
  if (!is_sentinel(v)) return v;
  const uint64_t t0 = wall_clock64();
  unsigned it = 0;
#pragma clang loop unroll(disable)
  while (is_sentinel(v)) {
    __builtin_amdgcn_s_sleep(1);
    v = ld_agent(p);
    if (is_sentinel(v) && (++it & 63u) == 0) {
      if (ld_agent(abort_flag)) return (T)__builtin_nan("");
      if (wall_clock64() - t0 > limit) {
        st_agent(abort_flag, 1);
        return (T)__builtin_nan("");
      }
    }
  }
  return v;
}

__device__ __forceinline__ double bcast_lane(double v, int j) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), j);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float bcast_lane(float v, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}

// task[8t ..]: kind (0 helper, 1 node), lo, s, r0, r1, node, has_ext, log2 G
template <class T, class TR, bool LOWER, bool DIAG>
__global__ __launch_bounds__(TREE_THREADS) void k_tree(const int* __restrict__ task, const int64_t* __restrict__ boff,
                                                       const int* __restrict__ erp, const int* __restrict__ ecol,
                                                       const T* __restrict__ eval, const T* __restrict__ blk,
                                                       const T* __restrict__ dinv, const TR* rhs, T* out, T* ext,
                                                       TR* reset_rhs, int* abort_flag, uint64_t limit) {
  extern __shared__ __align__(16) unsigned char tree_smem[];
  T* y = reinterpret_cast<T*>(tree_smem);
  const int* tk = task + 8 * (size_t)blockIdx.x;
  const int kind = tk[0], lo = tk[1], s = tk[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  if (kind == 0) {
    // ------------------------------------------------------------ helper
    // rows [r0, r1) of the node: ext[r] = rhs[r] - sum over entries outside
    // the node, G lanes per row, TREE_BATCH loads in flight per lane, pending
    // values polled as a group
    const int r0 = tk[3], r1 = tk[4], lg = tk[7];
    const int G = 1 << lg, per_wave = 64 >> lg;
    const int slot = lane >> lg, sub = lane & (G - 1);
    for (int rb = r0 + wave * per_wave; rb < r1; rb += (TREE_THREADS / 64) * per_wave) {
      const int r = rb + slot;
      const bool active = r < r1;
      T acc = (T)0;
      TR rh = (TR)0;
      if (active && sub == 0) rh = rhs[r];
      if (active) {
        const int q1 = erp[r + 1];
        for (int q = erp[r] + sub; q < q1; q += G * TREE_BATCH) {
          int c[TREE_BATCH];
          T v[TREE_BATCH], a[TREE_BATCH];
          unsigned need = 0;
#pragma unroll
          for (int u = 0; u < TREE_BATCH; ++u) {
            const int qq = q + u * G < q1 ? q + u * G : q1 - 1;
            c[u] = ecol[qq];
            a[u] = eval[qq];
            if (q + u * G < q1) need |= 1u << u;
          }
#pragma unroll
          for (int u = 0; u < TREE_BATCH; ++u) v[u] = ld_agent(out + c[u]);
#pragma unroll
          for (int u = 0; u < TREE_BATCH; ++u)
            if ((need >> u & 1u) && is_sentinel(v[u])) v[u] = tree_poll(out + c[u], abort_flag, limit);
#pragma unroll
          for (int u = 0; u < TREE_BATCH; ++u)
            if (need >> u & 1u) acc += a[u] * v[u];
        }
      }
      for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (active && sub == 0) {
        T e = (T)rh - acc;
        if (is_sentinel(e)) e = (T)__builtin_nan("");
        st_agent(ext + r, e);
        if (reset_rhs) reset_rhs[r] = sentinel_of<TR>(0);
      }
    }
    return;
  }

  // -------------------------------------------------------------- node
  const int has_ext = tk[6];
  const T* B = blk + boff[tk[5]];
  // the node's right-hand side: all loads issued first, pending ones polled
  // (s <= kTreeMaxRows, checked on the host)
  constexpr int YK = kTreeMaxRows / TREE_THREADS;
  {
    T v[YK];
#pragma unroll
    for (int k = 0; k < YK; ++k) {
      const int i = threadIdx.x + k * TREE_THREADS;
      if (i < s) v[k] = has_ext ? ld_agent(ext + lo + i) : (T)rhs[lo + i];
    }
#pragma unroll
    for (int k = 0; k < YK; ++k) {
      const int i = threadIdx.x + k * TREE_THREADS;
      if (i < s) {
        if (has_ext) {
          if (is_sentinel(v[k])) v[k] = tree_poll(ext + lo + i, abort_flag, limit);
          st_agent(ext + lo + i, sentinel_of<T>(0));
        } else if (reset_rhs) {
          reset_rhs[lo + i] = sentinel_of<TR>(0);
        }
        y[i] = v[k];
      }
    }
  }
  __syncthreads();
  const int np = (s + 63) / 64;
  for (int pi = 0; pi < np; ++pi) {
    // lower: panels top-down, columns left to right; upper: bottom-up,
    // columns right to left
    const int p0 = LOWER ? pi * 64 : std::max(0, s - (pi + 1) * 64);
    const int pw = LOWER ? std::min(64, s - p0) : (s - pi * 64) - p0;
    if (wave == 0) {
      const bool in = lane < pw;
      T yl = in ? y[p0 + lane] : (T)0;
      const T dl = DIAG ? (in ? dinv[lo + p0 + lane] : (T)0) : (T)1;
      // row p0 + lane of the panel: columns p0 .. p0 + pw - 1
      T b[64];
#pragma unroll
      for (int j = 0; j < 64; ++j) {
        const int jj = j < pw ? j : pw - 1;
        b[j] = B[(int64_t)(p0 + jj) * s + p0 + (in ? lane : 0)];
      }
      // columns in solve order; fully unrolled so that b[] stays in registers
      // (the bound pw is the same for the whole wave)
#pragma unroll
      for (int jr = 0; jr < 64; ++jr) {
        const int j = LOWER ? jr : 63 - jr;
        if (j < pw) {
          const T xj = bcast_lane(DIAG ? yl * dl : yl, j);
          yl -= b[j] * xj;  // zero in the other triangle: finished rows keep their value
        }
      }
      if (in) {
        T x = DIAG ? yl * dl : yl;
        if (is_sentinel(x)) x = (T)__builtin_nan("");
        y[p0 + lane] = x;
        st_agent(out + lo + p0 + lane, x);
      }
    }
    __syncthreads();
    // apply the panel to the rows still to be solved: one row per thread, the
    // panel's 64 entries of the row loaded together (a chain of dependent
    // loads would cost one memory round trip per column), then subtracted in
    // column order
    const int ra = LOWER ? p0 + pw : 0, rz = LOWER ? s : p0;
    for (int r = ra + threadIdx.x; r < rz; r += TREE_THREADS) {
      const T* col = B + (int64_t)p0 * s + r;
      T bb[64];
#pragma unroll
      for (int j = 0; j < 64; ++j) bb[j] = col[(int64_t)(j < pw ? j : pw - 1) * s];
      T acc = y[r];
#pragma unroll
      for (int j = 0; j < 64; ++j)
        if (j < pw) acc -= bb[j] * y[p0 + j];
      y[r] = acc;
    }
    __syncthreads();
  }
}

static uint64_t tree_limit_ticks() {
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
void launch_tree(const TreeSolve& ts, const void* rhs, bool rhs_is_f64, T* out, T* reset_rhs, T* ext, int* abort_flag,
                 hipStream_t s) {
  if (ts.ntasks == 0) return;
  constexpr bool F32 = sizeof(T) == 4;
  const T* ev = F32 ? (const T*)ts.eval32.p : (const T*)ts.eval.p;
  const T* bk = F32 ? (const T*)ts.blk32.p : (const T*)ts.blk.p;
  const T* di = F32 ? (const T*)ts.dinv32.p : (const T*)ts.dinv.p;
  const size_t lds = (size_t)ts.max_rows * sizeof(T);
  const uint64_t lim = tree_limit_ticks();
#define GMG_TREE(TR_, LO_, DG_, RHS_, RESET_)                                                                       \
  do {                                                                                                             \
    static bool attr = false;                                                                                      \
    if (!attr) {                                                                                                   \
      HIPCK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tree<T, TR_, LO_, DG_>),                          \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kTreeMaxRows * sizeof(double)))); \
      attr = true;                                                                                                 \
    }                                                                                                              \
    hipLaunchKernelGGL((k_tree<T, TR_, LO_, DG_>), dim3(ts.ntasks), dim3(TREE_THREADS), lds, s, ts.task.p,        \
                       ts.boff.p, ts.erp.p, ts.ecol.p, ev, bk, di, (const TR_*)RHS_, out, ext, RESET_, abort_flag,  \
                       lim);                                                                                       \
  } while (0)
#define GMG_TREE_RHS(TR_, RHS_, RESET_)                                        \
  do {                                                                         \
    if (ts.lower) {                                                            \
      if (ts.has_diag) GMG_TREE(TR_, true, true, RHS_, RESET_);                \
      else GMG_TREE(TR_, true, false, RHS_, RESET_);                           \
    } else {                                                                   \
      if (ts.has_diag) GMG_TREE(TR_, false, true, RHS_, RESET_);               \
      else GMG_TREE(TR_, false, false, RHS_, RESET_);                          \
    }                                                                          \
  } while (0)
  if (rhs_is_f64 && F32) GMG_TREE_RHS(double, rhs, (double*)nullptr);
  else GMG_TREE_RHS(T, rhs, reset_rhs);
#undef GMG_TREE_RHS
#undef GMG_TREE
  HIPCK(hipGetLastError());
}
template void launch_tree<double>(const TreeSolve&, const void*, bool, double*, double*, double*, int*, hipStream_t);
template void launch_tree<float>(const TreeSolve&, const void*, bool, float*, float*, float*, int*, hipStream_t);

}  // namespace gmg
