// Triangular solves over the nested-dissection tree (coarse ILUT factors).
//
// With the coarse unknowns numbered by nested dissection, an elimination only
// creates entries between a row and the rows of its own tree node or of the
// node's descendants (strictly lower part) or ancestors (strictly upper
// part).  So a lower solve can run bottom-up over the tree and an upper solve
// top-down: a node's rows are x = T^{-1} (rhs - E x_outside), where T is the
// node's diagonal block and the rows outside it that E refers to are final by
// then.  The diagonal blocks of separators are nearly dense after fill, and a
// substitution through one costs a dependent step per row; instead T^{-1} is
// formed once at setup (dense, column-major, zeros in the other triangle) and
// the solve applies it as a matrix-vector product, whose rows are independent
// and are split over several workgroups.
//
// One launch runs a whole solve as a list of tasks in tree order (lower:
// heights ascending; upper: descending).  For a node with terms outside it,
// helper tasks first compute rhs - (those terms) for slices of its rows,
// polling the published results of other nodes (value-as-flag, as in the
// sweeps), and publish them to a staging vector that doubles as its own
// ready flag; the node's slice tasks poll them, multiply, and publish their
// rows.  Every task waits only on earlier tasks and workgroups start in
// order, so the solve always makes progress; every wait is bounded.
#include <algorithm>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int TREE_THREADS = 256;
constexpr int TREE_BATCH = 8;   // helper loads in flight per lane
constexpr int TREE_MBATCH = 16; // inverse-block loads in flight per lane

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

// task[8t ..]: helper: 0, lo, s, r0, r1, node, 1, log2 G
//               slice:  1, lo, s, a, b, node, has_ext | log2 R << 1, slices
//               pair:   2, lo, s, node, lo', s', node', 0 (lower solves): two
//                       nodes of at most 64 rows without outside entries, one
//                       slice each, one per half of the workgroup (s' = 0:
//                       none), so that a tree's many leaves fit the workgroups
//                       resident at once
//
// nb > 1 solves nb right-hand sides in one launch: workgroup t * nb + c runs
// task t for column c, whose vectors (rhs, out, ext, reset_rhs) start at
// c * ld and whose node counters at c * nnode.  A task waits only on earlier
// tasks of its own column, which have lower workgroup indices.
template <class T, class TR, bool LOWER>
__global__ __launch_bounds__(TREE_THREADS) void k_tree(const int* __restrict__ task, const int64_t* __restrict__ boff,
                                                       const int* __restrict__ erp, const int* __restrict__ ecol,
                                                       const T* __restrict__ eval, const T* __restrict__ inv,
                                                       int* ncount, const TR* rhs, T* out, T* ext, TR* reset_rhs,
                                                       int* abort_flag, uint64_t limit, int nb, size_t ld, int nnode) {
  extern __shared__ __align__(16) unsigned char tree_smem[];
  T* y = reinterpret_cast<T*>(tree_smem);
  const int tix = blockIdx.x / nb;
  {
    const int col = blockIdx.x - tix * nb;
    rhs += col * ld;
    out += col * ld;
    ext += col * ld;
    if (reset_rhs) reset_rhs += col * ld;
    ncount += (size_t)col * nnode;
  }
  const int* tk = task + 8 * (size_t)tix;
  const int kind = tk[0];

  if (kind == 0) {
    // ------------------------------------------------------------ helper
    // rows [r0, r1) of the node: ext[r] = rhs[r] - sum over entries outside
    // the node, G lanes per row, TREE_BATCH loads in flight per lane, pending
    // values polled as a group
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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

  // ------------------------------------------------------- node slice
  // rows [a, b) of the node: x = Tinv[a:b, cols] y[cols], cols = [0, b)
  // (lower) or [a, s) (upper); R rows per slice, G = 256 / R column groups,
  // each thread one row and one group's columns, then a fixed-order sum of the
  // groups' partial sums
  // a pair task: threads [0, 128) take the first node, [128, 256) the second
  // (lower solves only: an upper solve's nodes without outside entries are
  // the few at the top of the tree)
  const bool pair = LOWER && kind == 2;
  const int half = pair ? (int)(threadIdx.x >> 7) : 0;
  const int tid = pair ? (int)(threadIdx.x & 127) : (int)threadIdx.x;
  const int nthr = pair ? TREE_THREADS / 2 : TREE_THREADS;
  const int lo = tk[1 + (pair ? 3 * half : 0)], s = tk[2 + (pair ? 3 * half : 0)];
  const int a = pair ? 0 : tk[3], b = pair ? s : tk[4], node = pair ? tk[3 + 3 * half] : tk[5];
  const int has_ext = pair ? 0 : tk[6] & 1, lgR = pair ? 6 : tk[6] >> 1, nsl = pair ? 1 : tk[7];
  const int j0 = LOWER ? 0 : a, j1 = LOWER ? b : s;
  __shared__ T part_all[TREE_THREADS];
  __shared__ int last_slice[2];
  T* part = part_all + half * (TREE_THREADS / 2);
  y += half * 64;  // a pair's second node: y holds at least 128 values then
  const int R = 1 << lgR, G = nthr >> lgR;
  const int rl = tid & (R - 1), cg = tid >> lgR;
  const int i = a + rl < b ? a + rl : a;
  const int ncol = j1 - j0, cw = (ncol + G - 1) / G;
  const int jg = j0 + cg * cw, jge = jg + cw < j1 ? jg + cw : j1;
  // the inverse of a triangular block is triangular: row i has no terms
  // past its diagonal (lower: columns <= i, upper: columns >= i), so each
  // thread reads only its row's side of the diagonal
  const int jb = LOWER ? jg : (jg > i ? jg : i);
  const int je = LOWER ? (jge < i + 1 ? jge : i + 1) : jge;
  const T* col = inv + boff[node] + i;  // column-major: Tinv[j][i] at j * s + i
  // the first batch of the block's entries does not depend on the
  // right-hand side: in flight while the inputs are awaited
  T m[TREE_MBATCH];
#pragma unroll
  for (int u = 0; u < TREE_MBATCH; ++u) m[u] = jb + u < je ? col[(int64_t)(jb + u) * s] : (T)0;
  // the slice's right-hand side: all loads issued first, pending ones polled
  // (s <= kTreeMaxRows, checked on the host)
  constexpr int YK = kTreeMaxRows / TREE_THREADS;
  {
    T v[YK];
#pragma unroll
    for (int k = 0; k < YK; ++k) {
      const int r = j0 + tid + k * nthr;
      if (r < j1) v[k] = has_ext ? ld_agent(ext + lo + r) : (T)rhs[lo + r];
    }
#pragma unroll
    for (int k = 0; k < YK; ++k) {
      const int r = j0 + tid + k * nthr;
      if (r < j1) {
        if (has_ext && is_sentinel(v[k])) v[k] = tree_poll(ext + lo + r, abort_flag, limit);
        y[r - j0] = v[k];
      }
    }
  }
  __syncthreads();
  T acc = (T)0;
#pragma unroll
  for (int u = 0; u < TREE_MBATCH; ++u)
    if (jb + u < je) acc += m[u] * y[jb + u - j0];
  for (int j = jb + TREE_MBATCH; j < je; j += TREE_MBATCH) {
#pragma unroll
    for (int u = 0; u < TREE_MBATCH; ++u) m[u] = j + u < je ? col[(int64_t)(j + u) * s] : (T)0;
#pragma unroll
    for (int u = 0; u < TREE_MBATCH; ++u)
      if (j + u < je) acc += m[u] * y[j + u - j0];
  }
  part[tid] = acc;
  __syncthreads();
  if (tid < R && a + tid < b) {
    T x = (T)0;
    for (int g = 0; g < G; ++g) x += part[g * R + tid];
    if (is_sentinel(x)) x = (T)__builtin_nan("");
    st_agent(out + lo + a + tid, x);
  }
  // the last slice of the node to get here resets what the slices read (the
  // counter is left at zero for the next solve).  Every slice has its inputs
  // in LDS by now; the count comes after the results are published so that
  // its round trip is not on the dependency chain, and a node of one slice
  // needs none.
  if (tid == 0) {
    bool last = true;
    if (nsl > 1) {
      const int t = atomicAdd(ncount + node, 1);
      last = t == nsl - 1;
      if (last) st_agent(ncount + node, 0);
    }
    last_slice[half] = last;
  }
  __syncthreads();
  if (last_slice[half]) {
    for (int r = tid; r < s; r += nthr) {
      if (has_ext) st_agent(ext + lo + r, sentinel_of<T>(0));
      else if (reset_rhs) reset_rhs[lo + r] = sentinel_of<TR>(0);
    }
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
                 hipStream_t s, int nb, size_t ld, int* ncount) {
  if (ts.ntasks == 0) return;
  if (nb < 1 || (int64_t)ts.ntasks * nb > 0x7fffffff) fail(GMG_ERR_INVALID_ARG, "tree solve: bad column count");
  if (nb > 1 && !ncount) fail(GMG_ERR_INVALID_ARG, "tree solve: columns need their own node counters");
  int* cnt = ncount ? ncount : ts.ncount.p;
  const int nnode = (int)ts.ncount.n;
  constexpr bool F32 = sizeof(T) == 4;
  const T* ev = F32 ? (const T*)ts.eval32.p : (const T*)ts.eval.p;
  const T* iv = F32 ? (const T*)ts.inv32.p : (const T*)ts.inv.p;
  const size_t lds = (size_t)std::max(ts.max_rows, 128) * sizeof(T);  // a pair task's two nodes: 2 x 64
  const uint64_t lim = tree_limit_ticks();
#define GMG_TREE(TR_, LO_, RHS_, RESET_)                                                                           \
  do {                                                                                                             \
    static bool attr = false;                                                                                      \
    if (!attr) {                                                                                                   \
      HIPCK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tree<T, TR_, LO_>),                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kTreeMaxRows * sizeof(double)))); \
      attr = true;                                                                                                 \
    }                                                                                                              \
    hipLaunchKernelGGL((k_tree<T, TR_, LO_>), dim3(ts.ntasks * nb), dim3(TREE_THREADS), lds, s, ts.task.p,        \
                       ts.boff.p, ts.erp.p, ts.ecol.p, ev, iv, cnt, (const TR_*)RHS_, out, ext, RESET_, abort_flag, \
                       lim, nb, ld, nnode);                                                                        \
  } while (0)
#define GMG_TREE_RHS(TR_, RHS_, RESET_)                \
  do {                                                 \
    if (ts.lower) GMG_TREE(TR_, true, RHS_, RESET_);   \
    else GMG_TREE(TR_, false, RHS_, RESET_);           \
  } while (0)
  if (rhs_is_f64 && F32) GMG_TREE_RHS(double, rhs, (double*)nullptr);
  else GMG_TREE_RHS(T, rhs, reset_rhs);
#undef GMG_TREE_RHS
#undef GMG_TREE
  HIPCK(hipGetLastError());
}
template void launch_tree<double>(const TreeSolve&, const void*, bool, double*, double*, double*, int*, hipStream_t,
                                  int, size_t, int*);
template void launch_tree<float>(const TreeSolve&, const void*, bool, float*, float*, float*, int*, hipStream_t, int,
                                 size_t, int*);

// ---------------------------------------------------------------- setup
// Inverse of a node's diagonal block T (unit diagonal, or diagonal 1/dinv):
// Tinv = T^{-1} by substitution on W columns of the identity at once (one
// workgroup per W-column chunk).  The chunk's unknowns X (rows x W) live in
// LDS; step k takes row k in elimination order (lower: ascending, upper:
// descending), finishes it, x_k = d_k X[k], stores it, and subtracts
// T[i][k] x_k from the rows i still to come.  The column of T that the next
// step needs is loaded during the current one and staged in LDS.
// itask[8t ..]: lo, s, c0, node, log2 W
template <bool LOWER, bool DIAG>
__global__ __launch_bounds__(TREE_THREADS) void k_tree_inv(const int* __restrict__ itask,
                                                           const int64_t* __restrict__ boff,
                                                           const double* __restrict__ blk,
                                                           const double* __restrict__ dinv, double* __restrict__ inv) {
  extern __shared__ __align__(16) unsigned char inv_smem[];
  const int* t = itask + 8 * (size_t)blockIdx.x;
  const int lo = t[0], s = t[1], c0 = t[2], node = t[3], lgW = t[4];
  const int W = 1 << lgW, RG = TREE_THREADS >> lgW;
  const int w = W < s - c0 ? W : s - c0;
  const int rbeg = LOWER ? c0 : 0, rend = LOWER ? s : c0 + w;
  const int nr = rend - rbeg;
  double* X = reinterpret_cast<double*>(inv_smem);  // X[(i - rbeg) * W + c]
  double* Tc = X + (size_t)nr * W;                   // two staged columns of T
  const double* Tb = blk + boff[node];
  double* M = inv + boff[node];
  const int c = threadIdx.x & (W - 1), g = threadIdx.x >> lgW;
  for (int q = threadIdx.x; q < nr * W; q += TREE_THREADS) X[q] = (rbeg + (q >> lgW) == c0 + (q & (W - 1))) ? 1.0 : 0.0;
  // rows of column k still to come: lower (k, rend), upper [rbeg, k)
  constexpr int PK = kTreeMaxRows / TREE_THREADS;
  auto row_at = [&](int k, int u) { return (LOWER ? k + 1 : rbeg) + (int)threadIdx.x + u * TREE_THREADS; };
  auto in_col = [&](int k, int i) { return LOWER ? i < rend : i < k; };
  {
    const int k = LOWER ? rbeg : rend - 1;
#pragma unroll
    for (int u = 0; u < PK; ++u) {
      const int i = row_at(k, u);
      if (in_col(k, i)) Tc[i - rbeg] = Tb[(int64_t)k * s + i];
    }
  }
  __syncthreads();
  for (int step = 0; step < nr; ++step) {
    const int k = LOWER ? rbeg + step : rend - 1 - step;
    const double* cur = Tc + (size_t)(step & 1) * nr;
    double* nxt = Tc + (size_t)((step + 1) & 1) * nr;
    // next column's loads in flight during this step's update
    const int kn = LOWER ? k + 1 : k - 1;
    const bool more = step + 1 < nr;
    double pre[PK];
#pragma unroll
    for (int u = 0; u < PK; ++u) {
      const int i = row_at(kn, u);
      pre[u] = (more && in_col(kn, i)) ? Tb[(int64_t)kn * s + i] : 0.0;
    }
    const double xk = (DIAG ? dinv[lo + k] : 1.0) * X[(k - rbeg) * W + c];
    if (g == 0 && c < w) M[(int64_t)(c0 + c) * s + k] = xk;
    if (LOWER) {
      for (int i = k + 1 + g; i < rend; i += RG) X[(i - rbeg) * W + c] -= cur[i - rbeg] * xk;
    } else {
      for (int i = rbeg + g; i < k; i += RG) X[(i - rbeg) * W + c] -= cur[i - rbeg] * xk;
    }
#pragma unroll
    for (int u = 0; u < PK; ++u) {
      const int i = row_at(kn, u);
      if (more && in_col(kn, i)) nxt[i - rbeg] = pre[u];
    }
    __syncthreads();
  }
}

size_t tree_inv_lds(int rows, int lgW) { return (size_t)rows * ((1 << lgW) + 2) * sizeof(double); }

int tree_inv_width(int rows) {
  // the widest chunk (at most 64 columns) whose LDS fits kTreeInvLds
  for (int lg = 6; lg > 0; --lg)
    if (tree_inv_lds(rows, lg) <= kTreeInvLds) return lg;
  return 0;
}

void launch_tree_invert(const TreeSolve& ts, const int* itask, int ntask, size_t lds, const double* blk,
                        const double* dinv, double* inv, hipStream_t s) {
  if (ntask == 0) return;
  if (lds > kTreeInvLds) fail(GMG_ERR_INVALID_ARG, "tree inverse: LDS request too large");
#define GMG_INV(LO_, DG_)                                                                                     \
  do {                                                                                                        \
    static bool attr = false;                                                                                 \
    if (!attr) {                                                                                              \
      HIPCK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tree_inv<LO_, DG_>),                         \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTreeInvLds));               \
      attr = true;                                                                                            \
    }                                                                                                         \
    hipLaunchKernelGGL((k_tree_inv<LO_, DG_>), dim3(ntask), dim3(TREE_THREADS), lds, s, itask, ts.boff.p, blk, \
                       dinv, inv);                                                                            \
  } while (0)
  if (ts.lower) {
    if (dinv) GMG_INV(true, true);
    else GMG_INV(true, false);
  } else {
    if (dinv) GMG_INV(false, true);
    else GMG_INV(false, false);
  }
#undef GMG_INV
  HIPCK(hipGetLastError());
}

// Setup: scatter a factor's rows (entries q in [rp[r] + skip, rp[r+1])) into
// the dense column-major diagonal blocks (entries inside the row's node) and
// the outside-entry lists (erp from the host's count of the same test), one
// thread per row.
__global__ void k_tree_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ v, int skip, const int* __restrict__ node_of,
                            const int* __restrict__ nlo, const int* __restrict__ nsz,
                            const int64_t* __restrict__ boff, const int* __restrict__ erp,
                            double* __restrict__ blk, int* __restrict__ ecol, double* __restrict__ eval) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int a = node_of[r], lo = nlo[a], sz = nsz[a];
  double* B = blk + boff[a];
  int e = erp[r];
  for (int q = rp[r] + skip; q < rp[r + 1]; ++q) {
    const int c = ci[q];
    if (node_of[c] == a) {
      B[(int64_t)(c - lo) * sz + (r - lo)] = v[q];
    } else {
      ecol[e] = c;
      eval[e] = v[q];
      ++e;
    }
  }
}

void launch_tree_fill(int n, const int* rp, const int* ci, const double* v, int skip, const int* node_of,
                      const int* nlo, const int* nsz, const int64_t* boff, const int* erp, double* blk, int* ecol,
                      double* eval, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tree_fill, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, v, skip, node_of, nlo, nsz, boff,
                     erp, blk, ecol, eval);
  HIPCK(hipGetLastError());
}

}  // namespace gmg
