// Finite-volume assembly of the convection-diffusion matrix A(kappa) and the
// gradients of a loss through the solve (dL/dkappa, dL/dA on the pattern).
//
// Discretisation of Eq. (pde): cell-centred finite volumes on [0,1]^dim,
// h = 1/n, row i + n j (+ n^2 k), rows scaled by the cell volume; harmonic
// face transmissibility T = 2 kc km / ((kc + km) h^2); Dirichlet faces y = 0, 1
// add 2 kc / h^2; Neumann faces add nothing; first-order upwind convection on
// face-averaged velocities.  The arithmetic order matches the generator that
// builds the same matrices on the host, so both give identical bits.
#include <mutex>

#include "gmg_internal.h"
#include "kcommon.h"

#pragma clang fp contract(off)

namespace gmg {

struct FvGeom {
  int n, dim;
  const double* fvel[3];
};

// face velocity of direction d at face index f (0..n) for the cell line (a, b)
// of the other coordinates; memory order of the face arrays is x fastest.
__device__ __forceinline__ double face_vel(const FvGeom& g, int d, const int* ijk, int f) {
  const int n = g.n;
  if (g.dim == 2) {
    if (d == 0) return g.fvel[0][(size_t)ijk[1] * (n + 1) + f];
    return g.fvel[1][(size_t)f * n + ijk[0]];
  }
  if (d == 0) return g.fvel[0][((size_t)ijk[2] * n + ijk[1]) * (n + 1) + f];
  if (d == 1) return g.fvel[1][((size_t)ijk[2] * (n + 1) + f) * n + ijk[0]];
  return g.fvel[2][((size_t)f * n + ijk[1]) * n + ijk[0]];
}

__device__ __forceinline__ int fv_row_count(int n, int dim, int c) {
  int ijk[3] = {c % n, (c / n) % n, dim == 3 ? c / (n * n) : 0};
  int k = 1;
  for (int d = 0; d < dim; ++d) k += (ijk[d] > 0) + (ijk[d] < n - 1);
  return k;
}

// cnt[c] = entries of row c for c < N, cnt[N] = 0 (N + 1 threads)
__global__ void k_fv_count(int n, int dim, int N, int* cnt) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N) cnt[c] = fv_row_count(n, dim, c);
  else if (c == N) cnt[N] = 0;
}

__global__ void k_fv_fill(FvGeom g, const double* __restrict__ kap, const int* __restrict__ rp,
                          int* __restrict__ ci, double* __restrict__ v, int N) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int n = g.n, dim = g.dim;
  const double h = 1.0 / n, h2 = h * h;
  int ijk[3] = {c % n, (c / n) % n, dim == 3 ? c / (n * n) : 0};
  const int stride[3] = {1, n, n * n};
  const double kc = kap[c];
  double diag = 0.0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool has_lo[3] = {false, false, false}, has_hi[3] = {false, false, false};
  for (int d = 0; d < dim; ++d) {
    const double Flo = face_vel(g, d, ijk, ijk[d]);
    const double Fhi = face_vel(g, d, ijk, ijk[d] + 1);
    const double out_hi = Fhi, out_lo = -Flo;
    double dint = 0.0;
    if (ijk[d] < n - 1) {
      const double km = kap[c + stride[d]];
      const double T = 2.0 * kc * km / ((kc + km) * h2);
      dint += T;
      has_hi[d] = true;
      hi[d] = (0.0 - T) + fmin(out_hi, 0.0) / h;
    }
    if (ijk[d] > 0) {
      const double km = kap[c - stride[d]];
      const double T = 2.0 * km * kc / ((km + kc) * h2);
      dint += T;
      has_lo[d] = true;
      lo[d] = (0.0 - T) + fmin(out_lo, 0.0) / h;
    }
    const double conv = fmax(out_hi, 0.0) / h + fmax(out_lo, 0.0) / h;
    diag += dint;
    diag += conv;
    if (d == 1) {
      if (ijk[1] == 0) diag += 2.0 * kc / h2;
      if (ijk[1] == n - 1) diag += 2.0 * kc / h2;
    }
  }
  int o = rp[c];
  for (int d = dim - 1; d >= 0; --d)
    if (has_lo[d]) { ci[o] = c - stride[d]; v[o] = lo[d]; ++o; }
  ci[o] = c;
  v[o] = diag;
  ++o;
  for (int d = 0; d < dim; ++d)
    if (has_hi[d]) { ci[o] = c + stride[d]; v[o] = hi[d]; ++o; }
}

// dL/dkappa_c = - sum_r [ sum over interior faces f of c of dT_f/dkappa_c
//   (lam_c - lam_m)(x_c - x_m) + sum over Dirichlet faces of (2/h^2) lam_c x_c ]
__global__ void k_fv_grad(int n, int dim, const double* __restrict__ kap, const double* __restrict__ lam,
                          const double* __restrict__ x, int nrhs, double* __restrict__ grad, int N) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double h = 1.0 / n, h2 = h * h;
  int ijk[3] = {c % n, (c / n) % n, dim == 3 ? c / (n * n) : 0};
  const int stride[3] = {1, n, n * n};
  const double kc = kap[c];
  double gsum = 0.0;
  for (int d = 0; d < dim; ++d) {
    for (int side = 0; side < 2; ++side) {
      const bool inside = side ? ijk[d] < n - 1 : ijk[d] > 0;
      if (inside) {
        const int m = side ? c + stride[d] : c - stride[d];
        const double km = kap[m];
        const double s = kc + km;
        const double dT = 2.0 * km * km / (s * s * h2);
        double acc = 0.0;
        for (int r = 0; r < nrhs; ++r)
          acc += (lam[(size_t)c * nrhs + r] - lam[(size_t)m * nrhs + r]) *
                 (x[(size_t)c * nrhs + r] - x[(size_t)m * nrhs + r]);
        gsum += dT * acc;
      } else if (d == 1) {
        double acc = 0.0;
        for (int r = 0; r < nrhs; ++r) acc += lam[(size_t)c * nrhs + r] * x[(size_t)c * nrhs + r];
        gsum += (2.0 / h2) * acc;
      }
    }
  }
  grad[c] = -gsum;
}

__global__ void k_pattern_grad(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ lam, const double* __restrict__ x, int nrhs,
                               double* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    double s = 0.0;
    for (int r = 0; r < nrhs; ++r) s += lam[(size_t)i * nrhs + r] * x[(size_t)j * nrhs + r];
    g[p] = -s;
  }
}

// Scratch of gmg_fv_assemble_noalloc: the block sums of its row-pointer scan
// (one int per SCAN_BS cells, plus the total), in a static array that every
// GPU the library runs on holds until the process ends.
static __device__ __align__(256) int scratch[GMG_FV_NOALLOC_SCRATCH_INTS];

// Device address of this GPU's copy of `scratch` (the array's name in host
// code is a host-side stand-in, not a device address): looked up once per
// device, with that device current.
static int* fv_scratch_ptr() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static int* ptr[kMaxDevices] = {};
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(GMG_ERR_INVALID_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = static_cast<int*>(p);
  }
  return ptr[dev];
}

}  // namespace gmg

using namespace gmg;

template <class F>
static gmg_status fv_guard(F&& f) {
  try {
    set_error_message("");
    return f();
  } catch (const Error& e) {
    set_error_message(e.msg);
    return e.code;
  }
}

extern "C" int64_t gmg_fv_nnz(int n, int dim) {
  if (n < 1 || (dim != 2 && dim != 3)) return -1;
  const int64_t N = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
  return (int64_t)(2 * dim + 1) * N - (int64_t)2 * dim * (N / n);
}

extern "C" gmg_status gmg_fv_assemble(int n, int dim, const double* kappa, const double* vel_x,
                                      const double* vel_y, const double* vel_z, int32_t* rowptr, int32_t* col,
                                      double* val, void* stream) {
  return fv_guard([&]() -> gmg_status {
    if (n < 1 || (dim != 2 && dim != 3) || !kappa || !vel_x || !vel_y || (dim == 3 && !vel_z) || !rowptr ||
        !col || !val)
      return GMG_ERR_INVALID_ARG;
    const int64_t N64 = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
    if (N64 >= (1LL << 31) / 8) return GMG_ERR_INVALID_ARG;
    const int N = (int)N64;
    hipStream_t s = (hipStream_t)stream;
    PoolStream pool_scope(s);  // declared before the buffers: they return to the cache first
    DBuf<int> cnt, tmp;
    cnt.alloc((size_t)N + 1);
    hipLaunchKernelGGL(k_fv_count, dim3((N + 1 + 255) / 256), dim3(256), 0, s, n, dim, N, cnt.p);
    launch_exclusive_scan_int(cnt.p, rowptr, N + 1, s, tmp);
    FvGeom g{n, dim, {vel_x, vel_y, dim == 3 ? vel_z : nullptr}};
    hipLaunchKernelGGL(k_fv_fill, dim3((N + 255) / 256), dim3(256), 0, s, g, kappa, rowptr, col, val, N);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return GMG_OK;
  });
}

extern "C" gmg_status gmg_fv_assemble_noalloc(int n, int dim, const double* kappa, const double* vel_x,
                                              const double* vel_y, const double* vel_z, int32_t* rowptr,
                                              int32_t* col, double* val, void* stream) {
  return fv_guard([&]() -> gmg_status {
    // every argument is checked before any device call
    if (n < 1 || (dim != 2 && dim != 3) || !kappa || !vel_x || !vel_y || (dim == 3 && !vel_z) || !rowptr ||
        !col || !val)
      return GMG_ERR_INVALID_ARG;
    const int64_t N64 = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
    if (N64 > GMG_FV_NOALLOC_MAX_CELLS) {
      set_error_message("gmg_fv_assemble_noalloc: " + std::to_string(N64) + " cells exceed the limit of " +
                        std::to_string((long long)GMG_FV_NOALLOC_MAX_CELLS));
      return GMG_ERR_INVALID_ARG;
    }
    static_assert((int64_t)GMG_FV_NOALLOC_SCRATCH_INTS * SCAN_BLOCK >= GMG_FV_NOALLOC_MAX_CELLS + 1 + SCAN_BLOCK,
                  "scratch holds one block sum per scan block plus the total");
    const int N = (int)N64;
    hipStream_t s = (hipStream_t)stream;
    int* bsum = fv_scratch_ptr();
    // the row counts go straight into rowptr and are scanned in place; the
    // scan's block sums live in the scratch array (every entry it reads is
    // written earlier in the same call, so nothing needs clearing)
    hipLaunchKernelGGL(k_fv_count, dim3((N + 1 + 255) / 256), dim3(256), 0, s, n, dim, N, rowptr);
    launch_exclusive_scan_int_ws(rowptr, rowptr, N + 1, bsum, s);
    FvGeom g{n, dim, {vel_x, vel_y, dim == 3 ? vel_z : nullptr}};
    hipLaunchKernelGGL(k_fv_fill, dim3((N + 255) / 256), dim3(256), 0, s, g, kappa, rowptr, col, val, N);
    HIPCK(hipGetLastError());
    return GMG_OK;
  });
}

extern "C" gmg_status gmg_fv_kappa_grad(int n, int dim, const double* kappa, const double* lambda,
                                        const double* x, int nrhs, double* grad, void* stream) {
  return fv_guard([&]() -> gmg_status {
    if (n < 1 || (dim != 2 && dim != 3) || !kappa || !lambda || !x || !grad || nrhs < 1)
      return GMG_ERR_INVALID_ARG;
    const int N = dim == 2 ? n * n : n * n * n;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fv_grad, dim3((N + 255) / 256), dim3(256), 0, s, n, dim, kappa, lambda, x, nrhs, grad, N);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return GMG_OK;
  });
}

extern "C" gmg_status gmg_pattern_grad(int64_t n, const int32_t* rowptr, const int32_t* col, const double* lambda,
                                       const double* x, int nrhs, double* gval, void* stream) {
  return fv_guard([&]() -> gmg_status {
    if (n < 1 || !rowptr || !col || !lambda || !x || !gval || nrhs < 1) return GMG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pattern_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int)n, rowptr, col,
                       lambda, x, nrhs, gval);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return GMG_OK;
  });
}
