// Dense exact coarse solve: the explicit inverse of A_c by blocked Gauss-Jordan
// elimination (no pivoting, the pivots of the no-pivot LU that the exact
// sparse factorisation also takes), then e_c = A_c^{-1} r_c as a dense
// matrix-vector product.  The matrix is row-major, padded to a multiple of 64
// rows and columns with the identity, so the padded matrix is
// blockdiag(A_c, I) and its inverse blockdiag(A_c^{-1}, I).
//
// One elimination step over the 64-wide block column K (D = A_KK^{-1}):
//   A_KK <- D;  A_Kj <- D A_Kj (j != K);  A_ij <- A_ij - A_iK A_Kj (i, j != K);
//   A_iK <- -A_iK D (i != K).
// FP64 matrix throughput equals the FP64 vector rate on this chip, so the
// rank-64 updates are register-tiled vector FMAs over 64x64 LDS tiles.
#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int DB = 64;  // block size of the elimination

__global__ void k_dense_scatter(int nc, int np, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, double* __restrict__ A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double* row = A + (size_t)i * np;
  if (i >= nc) {
    row[i] = 1.0;
    return;
  }
  for (int q = rp[i]; q < rp[i + 1]; ++q) row[ci[q]] += v[q];
}

// in-place Gauss-Jordan inverse of the 64x64 diagonal block K (one workgroup):
// thread t holds column t % 64, rows 16 (t / 64) .. +15 in registers; each
// elimination step publishes the pivot column and the scaled pivot row
// through LDS (double-buffered, two barriers a step)
__global__ __launch_bounds__(256) void k_gj_diag(int np, int K, double* __restrict__ A, int* __restrict__ bad) {
  __shared__ double colk[2][DB], rowk[2][DB];
  const int t = threadIdx.x, j = t & 63, g = t >> 6;
  double* blk = A + (size_t)K * DB * np + (size_t)K * DB;
  double a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) a[m] = blk[(size_t)(g * 16 + m) * np + j];
  // fully unrolled over k, so every register index is static and the
  // per-element cases are selects rather than branches
#pragma unroll
  for (int k = 0; k < DB; ++k) {
    const int buf = k & 1;
    if (j == k) {
#pragma unroll
      for (int m = 0; m < 16; ++m) colk[buf][g * 16 + m] = a[m];
    }
    __syncthreads();
    const double p = colk[buf][k];
    if (t == 0 && !(fabs(p) > 0.0 && fabs(p) < INFINITY)) *bad = 1;
    const double piv = 1.0 / p;
    if (g == (k >> 4)) {
      const double v = j != k ? a[k & 15] * piv : a[k & 15];
      a[k & 15] = v;
      rowk[buf][j] = v;
    }
    __syncthreads();
    const double rkj = rowk[buf][j];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int i = g * 16 + m;
      const double upd = a[m] - colk[buf][i] * rkj;
      const double colv = -a[m] * piv;
      const double rowv = j == k ? piv : a[m];
      a[m] = i != k ? (j != k ? upd : colv) : rowv;
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) blk[(size_t)(g * 16 + m) * np + j] = a[m];
}

// MODE 0: A_Kj <- D A_Kj (row panel, blockIdx.x = j block)
// MODE 1: A_iK <- -A_iK D (column panel, blockIdx.x = i block)
template <int MODE>
__global__ __launch_bounds__(256) void k_gj_panel(int np, int K, double* __restrict__ A) {
  const int b = blockIdx.x;
  if (b == K) return;
  __shared__ double d[DB][DB];
  __shared__ double x[DB][DB];
  const int t = threadIdx.x;
  const double* dk = A + (size_t)K * DB * np + (size_t)K * DB;
  double* tile = MODE == 0 ? A + (size_t)K * DB * np + (size_t)b * DB : A + (size_t)b * DB * np + (size_t)K * DB;
  for (int e = t; e < DB * DB; e += 256) {
    d[e / DB][e % DB] = dk[(size_t)(e / DB) * np + e % DB];
    x[e / DB][e % DB] = tile[(size_t)(e / DB) * np + e % DB];
  }
  __syncthreads();
  const int c = t & 63, r0 = (t >> 6) * 16;
  double acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  for (int k = 0; k < DB; ++k) {
    if (MODE == 0) {
      const double xk = x[k][c];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] += d[r0 + r][k] * xk;
    } else {
      const double dk_ = d[k][c];
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] += x[r0 + r][k] * dk_;
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) tile[(size_t)(r0 + r) * np + c] = MODE == 0 ? acc[r] : -acc[r];
}

// A_ij <- A_ij - A_iK A_Kj for i, j != K; grid (j block, i block).  Thread t
// accumulates a 4x4 block: rows t/16 + 16 r (r < 4), columns 4 (t % 16) .. +3;
// the A_iK tile's rows are padded to 65 so the four rows a wave reads at one
// k fall in distinct banks
__global__ __launch_bounds__(256) void k_gj_update(int np, int K, double* __restrict__ A) {
  const int jb = blockIdx.x, ib = blockIdx.y;
  if (ib == K || jb == K) return;
  __shared__ double p[DB][DB + 1];
  __shared__ double q[DB][DB];
  const int t = threadIdx.x;
  const double* pk = A + (size_t)ib * DB * np + (size_t)K * DB;
  const double* qk = A + (size_t)K * DB * np + (size_t)jb * DB;
  for (int e = t; e < DB * DB; e += 256) {
    p[e / DB][e % DB] = pk[(size_t)(e / DB) * np + e % DB];
    q[e / DB][e % DB] = qk[(size_t)(e / DB) * np + e % DB];
  }
  __syncthreads();
  const int cx = (t & 15) * 4, ry = t >> 4;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int k = 0; k < DB; ++k) {
    double pr[4], qc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) pr[r] = p[ry + 16 * r][k];
#pragma unroll
    for (int c = 0; c < 4; ++c) qc[c] = q[k][cx + c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += pr[r] * qc[c];
  }
  double* out = A + (size_t)ib * DB * np + (size_t)jb * DB;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) out[(size_t)(ry + 16 * r) * np + cx + c] -= acc[r][c];
}

void launch_dense_inverse(int nc, int np, const int* rp, const int* ci, const double* v, double* A, int* bad,
                          hipStream_t s) {
  if (nc <= 0) return;
  if (np % DB != 0 || np < nc) fail(GMG_ERR_INVALID_ARG, "dense inverse: padded size must be a multiple of 64 >= n_c");
  launch_fill_f64_bits(A, 0ULL, (size_t)np * np, s);
  hipLaunchKernelGGL(k_dense_scatter, dim3((np + 255) / 256), dim3(256), 0, s, nc, np, rp, ci, v, A);
  HIPCK(hipGetLastError());
  const int nb = np / DB;
  for (int K = 0; K < nb; ++K) {
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, s, np, K, A, bad);
    hipLaunchKernelGGL((k_gj_panel<0>), dim3(nb), dim3(256), 0, s, np, K, A);
    hipLaunchKernelGGL(k_gj_update, dim3(nb, nb), dim3(256), 0, s, np, K, A);
    hipLaunchKernelGGL((k_gj_panel<1>), dim3(nb), dim3(256), 0, s, np, K, A);
  }
  HIPCK(hipGetLastError());
}

// e = M r over the leading n x n part of the padded row-major M; one wave per row
template <class T>
__global__ __launch_bounds__(256) void k_dense_gemv(int n, int np, const T* __restrict__ M, const T* __restrict__ r,
                                                     T* __restrict__ e) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const T* m = M + (size_t)row * np;
  T acc = (T)0;
  for (int j = lane; j < n; j += 64) acc += m[j] * r[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) e[row] = acc;
}

template <class T>
void launch_dense_gemv(int n, int np, const T* M, const T* r, T* e, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_dense_gemv<T>), dim3((n + 3) / 4), dim3(256), 0, s, n, np, M, r, e);
  HIPCK(hipGetLastError());
}
template void launch_dense_gemv<double>(int, int, const double*, const double*, double*, hipStream_t);

// MT = M^T for the leading n x n block of padded row-major matrices (the
// adjoint cycle's coarse solve then reuses the product above): 64 x 64 tiles
// through LDS, read and written along rows
__global__ __launch_bounds__(256) void k_dense_transpose(int n, int np, const double* __restrict__ M,
                                                         double* __restrict__ MT) {
  __shared__ double tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4)
    if (r0 + r < n && c0 + tx < n) tile[r][tx] = M[(size_t)(r0 + r) * np + c0 + tx];
  __syncthreads();
  for (int c = ty; c < 64; c += 4)
    if (c0 + c < n && r0 + tx < n) MT[(size_t)(c0 + c) * np + r0 + tx] = tile[tx][c];
}

void launch_dense_transpose(int n, int np, const double* M, double* MT, hipStream_t s) {
  if (n <= 0) return;
  const unsigned t = (unsigned)((n + 63) / 64);
  hipLaunchKernelGGL(k_dense_transpose, dim3(t, t), dim3(256), 0, s, n, np, M, MT);
  HIPCK(hipGetLastError());
}
template void launch_dense_gemv<float>(int, int, const float*, const float*, float*, hipStream_t);

}  // namespace gmg
