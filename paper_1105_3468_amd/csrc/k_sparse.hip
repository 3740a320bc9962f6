// Sparse streaming kernels: SpMV, residual, restriction over aggregates,
// prolongation, CSR transpose, scans, fills.  All wave64, HBM-bound.
#include <algorithm>

#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(unsigned* p, unsigned v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned grid_for(size_t n, unsigned bs = 256, unsigned cap = 8192) {
  size_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

void launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  HIPCK(hipGetLastError());
}
void launch_fill_f64_bits(double* p, uint64_t bits, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, s, reinterpret_cast<uint64_t*>(p), bits, n);
  HIPCK(hipGetLastError());
}
void launch_fill_f32_bits(float* p, uint32_t bits, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, reinterpret_cast<unsigned*>(p), bits, n);
  HIPCK(hipGetLastError());
}

// ------------------------------------------------------------ validation
// flags[0]: structural error, flags[1]: non-finite value
__global__ void k_validate(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p0 = rp[i], p1 = rp[i + 1];
  bool bad = p1 < p0 || p0 < 0;
  bool diag = false, nonfin = false;
  if (!bad) {
    int prev = -1;
    for (int p = p0; p < p1; ++p) {
      int c = ci[p];
      if (c < 0 || c >= n || c <= prev) bad = true;
      if (c == i) diag = true;
      prev = c;
      if (!isfinite(v[p])) nonfin = true;
    }
  }
  if (bad || !diag) atomicOr(&flags[0], 1);
  if (nonfin) atomicOr(&flags[1], 1);
}
void launch_validate(int n, const int* rp, const int* ci, const double* v, int* flags, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_validate, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, v, flags);
  HIPCK(hipGetLastError());
}

__global__ void k_cast_f32(const double* __restrict__ x, float* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
void launch_cast_f32(const double* x, float* y, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
  HIPCK(hipGetLastError());
}

__global__ void k_gather_f64(const double* __restrict__ src, const int* __restrict__ idx,
                             double* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}
void launch_gather_f64(const double* src, const int* idx, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(n)), dim3(256), 0, s, src, idx, dst, n);
  HIPCK(hipGetLastError());
}

// Smoother in nested-dissection numbering: zp[k] = z[perm[k]] on the way in;
// t[perm[k]] = tp[k] on the way out, tp[k] <- sentinel (the next cycle's
// upper solve publishes into it again).
template <class T>
__global__ void k_perm_gather(int n, const int* __restrict__ perm, const double* __restrict__ z, T* __restrict__ zp) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) zp[k] = (T)z[perm[k]];
}
template <class T>
__global__ void k_perm_scatter(int n, const int* __restrict__ perm, T* __restrict__ tp, T* __restrict__ t) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    t[perm[k]] = tp[k];
    tp[k] = sentinel_of<T>(0);
  }
}
template <class T>
void launch_perm_gather(int n, const int* perm, const double* z, T* zp, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_perm_gather<T>, dim3(grid_for(n)), dim3(256), 0, s, n, perm, z, zp);
  HIPCK(hipGetLastError());
}
template <class T>
void launch_perm_scatter(int n, const int* perm, T* tp, T* t, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_perm_scatter<T>, dim3(grid_for(n)), dim3(256), 0, s, n, perm, tp, t);
  HIPCK(hipGetLastError());
}
template void launch_perm_gather<double>(int, const int*, const double*, double*, hipStream_t);
template void launch_perm_gather<float>(int, const int*, const double*, float*, hipStream_t);
template void launch_perm_scatter<double>(int, const int*, double*, double*, hipStream_t);
template void launch_perm_scatter<float>(int, const int*, float*, float*, hipStream_t);

// ------------------------------------------------------------------ SpMV
// One workgroup of 256 lanes owns 256 consecutive rows.  When the tile's
// entries fit in LDS, the lanes first stream the tile's (col, val) pairs with
// fully coalesced loads and store the products val * x[col] in LDS; then each
// lane sums its own row's products in column order.  Tiles with more entries
// than LDS holds fall back to one lane per row reading global memory.
// MODE 0: y = A x;  MODE 1: y = b - A x (b of type TB, converted to T).
constexpr int SPMV_ROWS = 256;
constexpr int SPMV_CAP = 4096;   // products held in LDS per tile
constexpr int SPMV_BATCH = 8;    // entries per lane whose loads are in flight together

template <class T, class TB, int MODE, int CAP>
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const T* __restrict__ v, const T* __restrict__ x,
                                              const TB* __restrict__ b, T* __restrict__ y) {
  __shared__ T prod[CAP];
  const int r0 = blockIdx.x * SPMV_ROWS;
  const int r1 = min(r0 + SPMV_ROWS, n);
  const int e0 = rp[r0], e1 = rp[r1];
  const int row = r0 + threadIdx.x;
  if (e1 - e0 <= CAP) {
    // a lane's entries e, e + 256, ... in batches of SPMV_BATCH: every column
    // index of the batch is loaded, then every x and value, then the products
    // (one round of dependent loads per batch instead of one per entry)
    for (int e = e0 + threadIdx.x; e < e1; e += 256 * SPMV_BATCH) {
      int c[SPMV_BATCH];
      T a[SPMV_BATCH], xv[SPMV_BATCH];
#pragma unroll
      for (int u = 0; u < SPMV_BATCH; ++u) c[u] = e + 256 * u < e1 ? ci[e + 256 * u] : -1;
#pragma unroll
      for (int u = 0; u < SPMV_BATCH; ++u) {
        a[u] = c[u] >= 0 ? v[e + 256 * u] : (T)0;
        xv[u] = c[u] >= 0 ? x[c[u]] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < SPMV_BATCH; ++u)
        if (c[u] >= 0) prod[e + 256 * u - e0] = a[u] * xv[u];
    }
    __syncthreads();
    if (row < r1) {
      T s = (T)0;
      const int a = rp[row] - e0, c = rp[row + 1] - e0;
      for (int k = a; k < c; ++k) s += prod[k];
      y[row] = MODE == 0 ? s : (T)b[row] - s;
    }
  } else if (row < r1) {
    T s = (T)0;
    for (int k = rp[row]; k < rp[row + 1]; ++k) s += v[k] * x[ci[k]];
    y[row] = MODE == 0 ? s : (T)b[row] - s;
  }
}

// The tile's capacity in LDS: 4096 products (32 KB in FP64: five
// workgroups per CU), or 2048 when every tile fits (16 KB: eight workgroups,
// the CU's wave limit, so more loads in flight).
int spmv_cap(int64_t max_tile_nnz) { return max_tile_nnz <= 2048 ? 2048 : 4096; }

template <class T, class TB, int MODE>
static void spmv_dispatch(int n, const int* rp, const int* ci, const T* v, const T* x, const TB* b, T* y, int cap,
                          hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid((n + SPMV_ROWS - 1) / SPMV_ROWS), blk(256);
  if (cap == 2048) hipLaunchKernelGGL((k_spmv<T, TB, MODE, 2048>), grid, blk, 0, s, n, rp, ci, v, x, b, y);
  else hipLaunchKernelGGL((k_spmv<T, TB, MODE, SPMV_CAP>), grid, blk, 0, s, n, rp, ci, v, x, b, y);
  HIPCK(hipGetLastError());
}

template <class T>
void launch_spmv(int n, const int* rp, const int* ci, const T* v, const T* x, T* y, hipStream_t s, int cap) {
  spmv_dispatch<T, T, 0>(n, rp, ci, v, x, (const T*)nullptr, y, cap, s);
}
template void launch_spmv<double>(int, const int*, const int*, const double*, const double*, double*, hipStream_t, int);
template void launch_spmv<float>(int, const int*, const int*, const float*, const float*, float*, hipStream_t, int);

void launch_residual(int n, const int* rp, const int* ci, const double* v, const double* x,
                     const double* b, double* r, hipStream_t s, int cap) {
  spmv_dispatch<double, double, 1>(n, rp, ci, v, x, b, r, cap, s);
}

template <class T>
void launch_resid_fine(int n, const int* rp, const int* ci, const T* v, const T* t, const double* z, T* r,
                       hipStream_t s, int cap) {
  spmv_dispatch<T, double, 1>(n, rp, ci, v, t, z, r, cap, s);
}
template void launch_resid_fine<double>(int, const int*, const int*, const double*, const double*, const double*, double*, hipStream_t, int);
template void launch_resid_fine<float>(int, const int*, const int*, const float*, const float*, const double*, float*, hipStream_t, int);

// ----------------------------------------------- restriction / prolongation
// rc[I] = sum over members k of G_I (ascending) of r[k]; reset[I] <- sentinel.
template <class T>
__global__ void k_restrict(int nc, const int* __restrict__ aptr, const int* __restrict__ amem,
                           const T* __restrict__ r, T* __restrict__ rc, T* __restrict__ reset,
                           uint64_t sent) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T s = (T)0;
  const int m0 = aptr[I], m1 = aptr[I + 1];
  // members in batches of eight: every index, then every value, then the
  // sums in member order (one round of dependent loads per batch)
  for (int m = m0; m < m1; m += 8) {
    int k[8];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) k[u] = m + u < m1 ? amem[m + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k[u] >= 0 ? r[k[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k[u] >= 0) s += v[u];
  }
  rc[I] = s;
  if (reset) reset[I] = sentinel_of<T>(sent);
}
template <class T>
void launch_restrict(int nc, const int* aptr, const int* amem, const T* r, T* rc, T* reset,
                     uint64_t sent, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_restrict<T>, dim3((nc + 255) / 256), dim3(256), 0, s, nc, aptr, amem, r, rc, reset, sent);
  HIPCK(hipGetLastError());
}
template void launch_restrict<double>(int, const int*, const int*, const double*, double*, double*, uint64_t, hipStream_t);
template void launch_restrict<float>(int, const int*, const int*, const float*, float*, float*, uint64_t, hipStream_t);

void launch_restrict_plain(int nc, const int* aptr, const int* amem, const double* z, double* bc,
                           double* reset, uint64_t sent, hipStream_t s) {
  launch_restrict<double>(nc, aptr, amem, z, bc, reset, sent, s);
}

// q[k] = t[k] + ec[agg[k]] in T, widened to double; with RESET t[k] <-
// sentinel (t is then the output of a sweep that polls for its values)
template <class T, bool RESET>
__global__ void k_prolong(int n, const int* __restrict__ agg, T* __restrict__ t, const T* __restrict__ ec,
                          double* __restrict__ q, uint64_t sent) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    T v = t[k] + ec[agg[k]];
    q[k] = (double)v;
    if (RESET) t[k] = sentinel_of<T>(sent);
  }
}
template <class T>
void launch_prolong(int n, const int* agg, T* t, const T* ec, double* q, uint64_t sent, hipStream_t s, bool reset_t) {
  if (n <= 0) return;
  if (reset_t) hipLaunchKernelGGL((k_prolong<T, true>), dim3(grid_for(n)), dim3(256), 0, s, n, agg, t, ec, q, sent);
  else hipLaunchKernelGGL((k_prolong<T, false>), dim3(grid_for(n)), dim3(256), 0, s, n, agg, t, ec, q, sent);
  HIPCK(hipGetLastError());
}
template void launch_prolong<double>(int, const int*, double*, const double*, double*, uint64_t, hipStream_t, bool);
template void launch_prolong<float>(int, const int*, float*, const float*, double*, uint64_t, hipStream_t, bool);

// adjoint residual: out[k] = z[k] - sum_l AT[k,l] * ec[agg[l]]
__global__ __launch_bounds__(256) void k_resid_adj(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ v, const int* __restrict__ agg,
                                                   const double* __restrict__ ec, const double* __restrict__ z,
                                                   double* __restrict__ out) {
  __shared__ double prod[SPMV_CAP];
  const int r0 = blockIdx.x * SPMV_ROWS;
  const int r1 = min(r0 + SPMV_ROWS, n);
  const int e0 = rp[r0], e1 = rp[r1];
  const int row = r0 + threadIdx.x;
  if (e1 - e0 <= SPMV_CAP) {
    for (int e = e0 + threadIdx.x; e < e1; e += 256) prod[e - e0] = v[e] * ec[agg[ci[e]]];
    __syncthreads();
    if (row < r1) {
      double s = 0.0;
      for (int k = rp[row] - e0; k < rp[row + 1] - e0; ++k) s += prod[k];
      out[row] = z[row] - s;
    }
  } else if (row < r1) {
    double s = 0.0;
    for (int k = rp[row]; k < rp[row + 1]; ++k) s += v[k] * ec[agg[ci[k]]];
    out[row] = z[row] - s;
  }
}
void launch_resid_adj(int n, const int* rp, const int* ci, const double* v, const int* agg,
                      const double* ec, const double* z, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_resid_adj, dim3((n + SPMV_ROWS - 1) / SPMV_ROWS), dim3(256), 0, s,
                     n, rp, ci, v, agg, ec, z, out);
  HIPCK(hipGetLastError());
}

// ------------------------------------------------------------------ scans
// Exclusive scan of n ints (out may alias in), three phases.
constexpr int SCAN_BS = 1024;

__global__ __launch_bounds__(SCAN_BS) void k_scan_block(const int* in, int* out, int n, int* __restrict__ bsum) {
  __shared__ int sh[SCAN_BS];
  int i = blockIdx.x * SCAN_BS + threadIdx.x;
  int v = i < n ? in[i] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BS; off <<= 1) {
    int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = sh[threadIdx.x] - v;
  if (threadIdx.x == SCAN_BS - 1) bsum[blockIdx.x] = sh[threadIdx.x];
}
__global__ void k_scan_sums(int* bsum, int nb) {
  // single thread: nb is small (n / 1024)
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < nb; ++b) { int t = bsum[b]; bsum[b] = acc; acc += t; }
    bsum[nb] = acc;
  }
}
__global__ void k_scan_add(int* out, int n, const int* bsum) {
  int i = blockIdx.x * SCAN_BS + threadIdx.x;
  if (i < n) out[i] += bsum[blockIdx.x];
}

static_assert(SCAN_BS == SCAN_BLOCK, "scan block size");

// bsum: caller's workspace of at least n / SCAN_BS + 2 ints
void launch_exclusive_scan_int_ws(const int* in, int* out, int n, int* bsum, hipStream_t s) {
  if (n <= 0) return;
  int nb = (n + SCAN_BS - 1) / SCAN_BS;
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(SCAN_BS), 0, s, in, out, n, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_BS), 0, s, out, n, bsum);
  HIPCK(hipGetLastError());
}

void launch_exclusive_scan_int(const int* in, int* out, int n, hipStream_t s, DBuf<int>& tmp) {
  if (n <= 0) return;
  int nb = (n + SCAN_BS - 1) / SCAN_BS;
  if ((int)tmp.n < nb + 1) tmp.alloc(nb + 1);
  launch_exclusive_scan_int_ws(in, out, n, tmp.p, s);
}

// ---------------------------------------------------------------- transpose
__global__ void k_count_cols(int64_t nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[p]], 1);
}
__global__ void k_scatter_t(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                            int* __restrict__ fill, int* __restrict__ tci, int* __restrict__ tsrc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    int q = atomicAdd(&fill[ci[p]], 1);
    tci[q] = i;
    tsrc[q] = p;
  }
}
// per transposed row: insertion sort of (tci, tsrc) by tci (keys unique)
__global__ void k_sort_rows(int m, const int* __restrict__ trp, int* __restrict__ tci, int* __restrict__ tsrc) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  int a = trp[j], b = trp[j + 1];
  for (int p = a + 1; p < b; ++p) {
    int kc = tci[p], ks = tsrc[p];
    int q = p - 1;
    while (q >= a && tci[q] > kc) { tci[q + 1] = tci[q]; tsrc[q + 1] = tsrc[q]; --q; }
    tci[q + 1] = kc;
    tsrc[q + 1] = ks;
  }
}

void transpose_csr(int n, int m, int64_t nnz, const int* rp, const int* ci, const double* v,
                   DBuf<int>& trp, DBuf<int>& tci, DBuf<double>* tv, DBuf<int>* tsrc_out, hipStream_t s) {
  trp.alloc((size_t)m + 1);
  tci.alloc(nnz > 0 ? nnz : 1);
  DBuf<int> tsrc_local;
  DBuf<int>& tsrc = tsrc_out ? *tsrc_out : tsrc_local;
  tsrc.alloc(nnz > 0 ? nnz : 1);
  DBuf<int> cnt, tmp;
  cnt.alloc((size_t)m + 1);
  HIPCK(hipMemsetAsync(cnt.p, 0, sizeof(int) * ((size_t)m + 1), s));
  if (nnz > 0)
    hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, ci, cnt.p);
  launch_exclusive_scan_int(cnt.p, trp.p, m + 1, s, tmp);
  DBuf<int> fill;
  fill.alloc((size_t)m + 1);
  d2d(fill.p, trp.p, (size_t)m + 1, s);
  if (n > 0)
    hipLaunchKernelGGL(k_scatter_t, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, fill.p, tci.p, tsrc.p);
  if (m > 0)
    hipLaunchKernelGGL(k_sort_rows, dim3((m + 255) / 256), dim3(256), 0, s, m, trp.p, tci.p, tsrc.p);
  HIPCK(hipGetLastError());
  if (tv) {
    tv->alloc(nnz > 0 ? nnz : 1);
    launch_gather_f64(v, tsrc.p, tv->p, nnz, s);
  }
  HIPCK(hipStreamSynchronize(s));   // temporaries are freed on return
}

}  // namespace gmg
