// Kernels of the multi-right-hand-side solve: one launch processes up to
// BATCH_MAX columns, so the matrix, the aggregates and the factors are read
// once for all of them.  A batch of vectors is column-major: column c starts
// at base + c * ld (ld a multiple of 64 elements, so every column is aligned
// like a single vector).
//
//   k_spmm           y_c = A x_c, or y_c = b_c - A x_c (the FGMRES residual),
//                    or y_c = z_c - A^T P e_c (the adjoint cycle's residual)
//   k_restrict_cols  r_c = P^T z_c (members in ascending order)
//   k_prolong_cols   q_c = t_c + P e_c
//   k_cols_from_rows / k_rows_from_cols: between the caller's (N, nrhs)
//                    row-major arrays and the column-major batch
#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int BROWS = 256;    // rows per workgroup of the sparse products
constexpr int BCAP = 3072;    // (column, value) pairs of a tile staged in LDS

// One workgroup owns BROWS consecutive rows.  When the tile's entries fit in
// LDS they are first staged there with coalesced loads; then each lane runs
// its own row, reading the entry once and the nb columns' values of x at that
// entry (consecutive lanes hold consecutive rows, so for fixed column and
// entry position the gathers are nearly contiguous).
// MODE 0: y = A x; 1: y = b - A x; 2: y = b - A (P e), x indexed through agg.
template <class T, class TB, int MODE>
__global__ __launch_bounds__(BROWS) void k_spmm(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const T* __restrict__ v, const int* __restrict__ agg,
                                                const T* __restrict__ x, size_t ldx, const TB* __restrict__ b,
                                                size_t ldb, T* __restrict__ y, size_t ldy, int nb) {
  __shared__ int sc[BCAP];
  __shared__ T sv[BCAP];
  const int r0 = blockIdx.x * BROWS;
  const int r1 = min(r0 + BROWS, n);
  const int e0 = rp[r0], e1 = rp[r1];
  const int row = r0 + threadIdx.x;
  const bool staged = e1 - e0 <= BCAP;
  if (staged) {
    for (int e = e0 + threadIdx.x; e < e1; e += BROWS) {
      sc[e - e0] = ci[e];
      sv[e - e0] = v[e];
    }
    __syncthreads();
  }
  if (row >= r1) return;
  T acc[BATCH_MAX];
#pragma unroll
  for (int c = 0; c < BATCH_MAX; ++c) acc[c] = (T)0;
  const int p0 = rp[row], p1 = rp[row + 1];
  for (int p = p0; p < p1; ++p) {
    int j;
    T a;
    if (staged) {
      j = sc[p - e0];
      a = sv[p - e0];
    } else {
      j = ci[p];
      a = v[p];
    }
    if (MODE == 2) j = agg[j];
    T xv[BATCH_MAX];
#pragma unroll
    for (int c = 0; c < BATCH_MAX; ++c) xv[c] = c < nb ? x[c * ldx + j] : (T)0;
#pragma unroll
    for (int c = 0; c < BATCH_MAX; ++c) acc[c] += a * xv[c];
  }
#pragma unroll
  for (int c = 0; c < BATCH_MAX; ++c)
    if (c < nb) y[c * ldy + row] = MODE == 0 ? acc[c] : (T)b[c * ldb + row] - acc[c];
}

template <class T, class TB, int MODE>
static void spmm_launch(int n, const int* rp, const int* ci, const T* v, const int* agg, const T* x, size_t ldx,
                        const TB* b, size_t ldb, T* y, size_t ldy, int nb, hipStream_t s) {
  if (n <= 0) return;
  if (nb < 1 || nb > BATCH_MAX) fail(GMG_ERR_INVALID_ARG, "spmm: bad column count");
  hipLaunchKernelGGL((k_spmm<T, TB, MODE>), dim3((n + BROWS - 1) / BROWS), dim3(BROWS), 0, s, n, rp, ci, v, agg, x,
                     ldx, b, ldb, y, ldy, nb);
  HIPCK(hipGetLastError());
}

template <class T>
void launch_spmm(int n, const int* rp, const int* ci, const T* v, const T* x, size_t ldx, T* y, size_t ldy, int nb,
                 hipStream_t s) {
  spmm_launch<T, T, 0>(n, rp, ci, v, nullptr, x, ldx, (const T*)nullptr, 0, y, ldy, nb, s);
}
template void launch_spmm<double>(int, const int*, const int*, const double*, const double*, size_t, double*, size_t,
                                  int, hipStream_t);
template void launch_spmm<float>(int, const int*, const int*, const float*, const float*, size_t, float*, size_t,
                                 int, hipStream_t);

void launch_residual_cols(int n, const int* rp, const int* ci, const double* v, const double* x, size_t ldx,
                          const double* b, size_t ldb, double* r, size_t ldr, int nb, hipStream_t s) {
  spmm_launch<double, double, 1>(n, rp, ci, v, nullptr, x, ldx, b, ldb, r, ldr, nb, s);
}

void launch_resid_adj_cols(int n, const int* rp, const int* ci, const double* v, const int* agg, const double* ec,
                           size_t ldc, const double* z, size_t ldz, double* out, size_t ldo, int nb, hipStream_t s) {
  spmm_launch<double, double, 2>(n, rp, ci, v, agg, ec, ldc, z, ldz, out, ldo, nb, s);
}

// r_c = z_c - A t_c over the column batch (t in the cycle's precision T, z
// in FP64): the fine residual of the smoothed iterate
template <class T>
void launch_resid_fine_cols(int n, const int* rp, const int* ci, const T* v, const T* t, size_t ldt, const double* z,
                            size_t ldz, T* r, size_t ldr, int nb, hipStream_t s) {
  spmm_launch<T, double, 1>(n, rp, ci, v, nullptr, t, ldt, z, ldz, r, ldr, nb, s);
}
template void launch_resid_fine_cols<double>(int, const int*, const int*, const double*, const double*, size_t,
                                             const double*, size_t, double*, size_t, int, hipStream_t);
template void launch_resid_fine_cols<float>(int, const int*, const int*, const float*, const float*, size_t,
                                            const double*, size_t, float*, size_t, int, hipStream_t);

// rc_c[I] = sum over members (ascending) of z_c[k]; reset_c[I] <- sentinel
// (column blockIdx.y)
template <class T, class TZ>
__global__ void k_restrict_cols(int nc, const int* __restrict__ aptr, const int* __restrict__ amem,
                                const TZ* __restrict__ z, size_t ldz, T* __restrict__ rc, T* __restrict__ reset,
                                size_t ldc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  z += blockIdx.y * ldz;
  T s = (T)0;
  for (int m = aptr[I]; m < aptr[I + 1]; ++m) s += (T)z[amem[m]];
  rc[blockIdx.y * ldc + I] = s;
  if (reset) reset[blockIdx.y * ldc + I] = sentinel_of<T>(0);
}
void launch_restrict_cols(int nc, const int* aptr, const int* amem, const double* z, size_t ldz, double* rc,
                          double* reset, size_t ldc, int nb, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL((k_restrict_cols<double, double>), dim3((nc + 255) / 256, nb), dim3(256), 0, s, nc, aptr, amem, z,
                     ldz, rc, reset, ldc);
  HIPCK(hipGetLastError());
}
template <class T>
void launch_restrict_cols_t(int nc, const int* aptr, const int* amem, const T* r, size_t ldr, T* rc, T* reset,
                            size_t ldc, int nb, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL((k_restrict_cols<T, T>), dim3((nc + 255) / 256, nb), dim3(256), 0, s, nc, aptr, amem, r, ldr, rc,
                     reset, ldc);
  HIPCK(hipGetLastError());
}
template void launch_restrict_cols_t<double>(int, const int*, const int*, const double*, size_t, double*, double*,
                                             size_t, int, hipStream_t);
template void launch_restrict_cols_t<float>(int, const int*, const int*, const float*, size_t, float*, float*, size_t,
                                            int, hipStream_t);

// q_c[k] = t_c[k] + ec_c[agg[k]] (in T, widened); t_c[k] <- sentinel
template <class T>
__global__ void k_prolong_cols(int n, const int* __restrict__ agg, T* __restrict__ t, size_t ldt,
                               const T* __restrict__ ec, size_t ldc, double* __restrict__ q, size_t ldq) {
  t += blockIdx.y * ldt;
  ec += blockIdx.y * ldc;
  q += blockIdx.y * ldq;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const T val = t[k] + ec[agg[k]];
    q[k] = (double)val;
    t[k] = sentinel_of<T>(0);
  }
}
template <class T>
void launch_prolong_cols(int n, const int* agg, T* t, size_t ldt, const T* ec, size_t ldc, double* q, size_t ldq,
                         int nb, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
  hipLaunchKernelGGL(k_prolong_cols<T>, dim3(g, nb), dim3(256), 0, s, n, agg, t, ldt, ec, ldc, q, ldq);
  HIPCK(hipGetLastError());
}
template void launch_prolong_cols<double>(int, const int*, double*, size_t, const double*, size_t, double*, size_t,
                                          int, hipStream_t);
template void launch_prolong_cols<float>(int, const int*, float*, size_t, const float*, size_t, double*, size_t, int,
                                         hipStream_t);

// out_c[i] = X[i * nrhs + c0 + c] for c < nb (column blockIdx.y), and back
__global__ void k_cols_from_rows(const double* __restrict__ X, int nrhs, int c0, double* __restrict__ out, size_t ld,
                                 int64_t n) {
  const int c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[c * ld + i] = X[i * nrhs + c0 + c];
}
__global__ void k_rows_from_cols(double* __restrict__ X, int nrhs, int c0, const double* __restrict__ in, size_t ld,
                                 int64_t n) {
  const int c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i * nrhs + c0 + c] = in[c * ld + i];
}
void launch_cols_from_rows(const double* X, int nrhs, int c0, double* out, size_t ld, int64_t n, int nb,
                           hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_cols_from_rows, dim3(g, nb), dim3(256), 0, s, X, nrhs, c0, out, ld, n);
  HIPCK(hipGetLastError());
}
void launch_rows_from_cols(double* X, int nrhs, int c0, const double* in, size_t ld, int64_t n, int nb,
                           hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_rows_from_cols, dim3(g, nb), dim3(256), 0, s, X, nrhs, c0, in, ld, n);
  HIPCK(hipGetLastError());
}

}  // namespace gmg
