// Krylov-subspace vector kernels of FGMRES: block multi-dot products, the two
// fused classical Gram-Schmidt passes (CGS2), norms, scaling and the solution
// update.  Reductions are deterministic: every block writes its partial sums
// in a fixed order and the last block to finish adds the partials in block
// order (no floating-point atomics), so repeated runs are bitwise identical.
// The partials are published like the sweeps' results: relaxed agent-scope
// stores into a buffer reset to a NaN sentinel, polled by the last block,
// which resets them again.  No fence is needed; an agent-scope fence writes
// the whole L2 back and cost ~40 us per launch here.
#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

constexpr int KB = 256;          // threads per block
constexpr int KGRID = 512;       // blocks of the reduction kernels
constexpr int KMAX = 32;         // vectors per fused register-resident pass
constexpr int KLDS = 2048;       // vectors per LDS-staged pass (longest basis)
// many-vector passes (a basis longer than KMAX)
constexpr int MKB = 512;          // threads per block
constexpr int MROWS = 64;         // rows per chunk (two per thread)
constexpr int MG = MKB / (MROWS / 2);  // vector groups per block
constexpr int MGRID = 256;        // blocks (one per CU)
constexpr int MMAX = 384;         // longest basis they take (24 vectors per thread group)
constexpr int MPARTS = 32;        // thread groups adding the block partials of one vector
constexpr int MPIPE = 16;         // up to this many vectors per thread, the next chunk is loaded early
constexpr int MSTR = MMAX + 8;    // stride of a block's row of partials (one extra slot for a norm)

// Keeps the machine scheduler from sinking the loads issued above it into the
// arithmetic below: without it the compiler reuses one register pair for all
// K basis loads of an element and waits for each in turn.
#define ALL_LOADS_ISSUED() __builtin_amdgcn_sched_barrier(0)

template <int K>
__device__ __forceinline__ void block_reduce_store(double (&acc)[K], int kcount, double* partial,
                                                   unsigned* counter, double* result) {
  __shared__ double sh[KB / 64][K];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kcount) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KB / 64; ++w) s += sh[w][threadIdx.x];
    if (is_sentinel(s)) s = __builtin_nan("");
    st_agent(&partial[(size_t)blockIdx.x * KMAX + threadIdx.x], s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(counter, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) {
    // all threads take part: thread t adds blocks part, part + NP, ... of
    // vector k (t = part * K + k), then thread k adds the NP parts in order
    constexpr int NP = KB / K;
    __shared__ double sh2[NP][K];
    const int k = threadIdx.x % K, part = threadIdx.x / K;
    if (part < NP) {
      double s = 0.0;
      if (k < kcount) {
        // 16 partials in flight at a time, added in block order; a partial
        // not yet visible is polled (its block stored it before counting)
        double* pp = partial + k;
        for (unsigned b0 = part; b0 < gridDim.x; b0 += 16 * NP) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const unsigned b = b0 + u * NP;
            v[u] = b < gridDim.x ? ld_agent(pp + (size_t)b * KMAX) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const unsigned b = b0 + u * NP;
            if (b < gridDim.x) {
              unsigned spins = 0;
#pragma clang loop unroll(disable)
              while (is_sentinel(v[u])) {
                if (++spins > (1u << 22)) { v[u] = __builtin_nan(""); break; }  // bounded
                __builtin_amdgcn_s_sleep(1);
                v[u] = ld_agent(pp + (size_t)b * KMAX);
              }
              s += v[u];
              st_agent(pp + (size_t)b * KMAX, sentinel_of<double>(0));
            }
          }
        }
      }
      sh2[part][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kcount) {
      double s = 0.0;
      for (int q = 0; q < NP; ++q) s += sh2[q][threadIdx.x];
      result[threadIdx.x] = s;
    }
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// result[k] = sum_i V[k][i] w[i], k < K.  The vector count is a compile-time
// constant so the K loads of an element are unconditional and all in flight.
// Batched forms (several independent FGMRES recurrences per launch): column
// c = blockIdx.y works on V + c * vcol, w + c * wcol and writes result +
// c * rcol, with its own block partials and counter.
#define KRYLOV_COLUMN()                                   \
  do {                                                    \
    const size_t col_ = blockIdx.y;                       \
    V += col_ * vcol;                                     \
    w += col_ * wcol;                                     \
    result += col_ * rcol;                                \
    partial += col_ * (size_t)KGRID * KMAX;               \
    counter += col_;                                      \
  } while (0)

template <int K>
__global__ __launch_bounds__(KB) void k_multidot(const double* __restrict__ V, size_t ld, int kc,
                                                 const double* __restrict__ w, int64_t n, double* partial,
                                                 unsigned* counter, double* result, size_t vcol, size_t wcol,
                                                 size_t rcol) {
  KRYLOV_COLUMN();
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    const double wi = w[i];
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = V[k * ld + i];
    ALL_LOADS_ISSUED();
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k] * wi;
  }
  block_reduce_store<K>(acc, kc, partial, counter, result);
}

// w <- w - sum_k h[k] V[k]; result[k] = V[k] . w_new
template <int K>
__global__ __launch_bounds__(KB) void k_update_dot(const double* __restrict__ V, size_t ld, int kc,
                                                   const double* __restrict__ h, double* __restrict__ w,
                                                   int64_t n, double* partial, unsigned* counter,
                                                   double* result, size_t vcol, size_t wcol, size_t rcol,
                                                   size_t hcol) {
  KRYLOV_COLUMN();
  h += blockIdx.y * hcol;
  double acc[K], hk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) { acc[k] = 0.0; hk[k] = h[k]; }
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    double v[K];
    double s = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = V[k * ld + i];
    ALL_LOADS_ISSUED();
#pragma unroll
    for (int k = 0; k < K; ++k) s -= hk[k] * v[k];
    w[i] = s;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k] * s;
  }
  block_reduce_store<K>(acc, kc, partial, counter, result);
}

// w <- w - sum_k h[k] V[k]; result[0] = ||w_new||^2
template <int K>
__global__ __launch_bounds__(KB) void k_update_norm(const double* __restrict__ V, size_t ld, int kc,
                                                    const double* __restrict__ h, double* __restrict__ w,
                                                    int64_t n, double* partial, unsigned* counter,
                                                    double* result, size_t vcol, size_t wcol, size_t rcol,
                                                    size_t hcol) {
  KRYLOV_COLUMN();
  h += blockIdx.y * hcol;
  double acc[1] = {0.0}, hk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) hk[k] = h[k];
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    double v[K];
    double s = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = V[k * ld + i];
    ALL_LOADS_ISSUED();
#pragma unroll
    for (int k = 0; k < K; ++k) s -= hk[k] * v[k];
    w[i] = s;
    acc[0] += s * s;
  }
  block_reduce_store<1>(acc, 1, partial, counter, result);
}

void red_init(RedWork& rw, hipStream_t s) {
  rw.blocks = KGRID;
  rw.partial.alloc((size_t)KGRID * KMAX * KCOLS);
  rw.counter.alloc(KCOLS);
  rw.result.alloc(2 * KLDS + 8);
  rw.mpart.alloc((size_t)MGRID * MSTR);
  launch_fill_u32(rw.counter.p, 0u, KCOLS, s);
  launch_fill_f64_bits(rw.partial.p, SENT64, (size_t)KGRID * KMAX * KCOLS, s);
}

// Back to the state red_init leaves (every partial the sentinel, counters
// zero), after a reduction may have given up on a partial (its bounded wait
// ran out): a partial that lands later must not be read by the next one.
void red_reset(RedWork& rw, hipStream_t s) {
  launch_fill_u32(rw.counter.p, 0u, KCOLS, s);
  launch_fill_f64_bits(rw.partial.p, SENT64, (size_t)KGRID * KMAX * KCOLS, s);
}

static unsigned red_grid(int64_t n) {
  int64_t g = (n + KB - 1) / KB;
  if (g > KGRID) g = KGRID;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// launch KERNEL<kc> for 1 <= kc <= 32
#define GMG_K4(KERNEL, B, ...)                                           \
  case B + 1: hipLaunchKernelGGL(KERNEL<B + 1>, __VA_ARGS__); break;    \
  case B + 2: hipLaunchKernelGGL(KERNEL<B + 2>, __VA_ARGS__); break;    \
  case B + 3: hipLaunchKernelGGL(KERNEL<B + 3>, __VA_ARGS__); break;    \
  case B + 4: hipLaunchKernelGGL(KERNEL<B + 4>, __VA_ARGS__); break;
#define GMG_DISPATCH_K(kc, KERNEL, ...)                                                                   \
  do {                                                                                                    \
    switch (kc) {                                                                                         \
      GMG_K4(KERNEL, 0, __VA_ARGS__) GMG_K4(KERNEL, 4, __VA_ARGS__) GMG_K4(KERNEL, 8, __VA_ARGS__)         \
      GMG_K4(KERNEL, 12, __VA_ARGS__) GMG_K4(KERNEL, 16, __VA_ARGS__) GMG_K4(KERNEL, 20, __VA_ARGS__)      \
      GMG_K4(KERNEL, 24, __VA_ARGS__) GMG_K4(KERNEL, 28, __VA_ARGS__)                                     \
      default: fail(GMG_ERR_INVALID_ARG, "vector count out of range");                                    \
    }                                                                                                     \
  } while (0)

static void check_cols(const BatchCols& bc) {
  if (bc.nb < 1 || bc.nb > KCOLS) fail(GMG_ERR_INVALID_ARG, "Krylov kernels: bad column count");
}
void launch_multidot(const double* V, size_t ld, int k, const double* w, int64_t n, RedWork& rw,
                     double* result, hipStream_t s, const BatchCols& bc) {
  if (k < 1 || k > KMAX) fail(GMG_ERR_INVALID_ARG, "multidot: bad vector count");
  check_cols(bc);
  GMG_DISPATCH_K(k, k_multidot, dim3(red_grid(n), bc.nb), dim3(KB), 0, s, V, ld, k, w, n, rw.partial.p,
                 rw.counter.p, result, bc.vcol, bc.wcol, bc.rcol);
  HIPCK(hipGetLastError());
}
void launch_update_dot(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, RedWork& rw,
                       double* result, hipStream_t s, const BatchCols& bc) {
  if (k < 1 || k > KMAX) fail(GMG_ERR_INVALID_ARG, "update_dot: bad vector count");
  check_cols(bc);
  GMG_DISPATCH_K(k, k_update_dot, dim3(red_grid(n), bc.nb), dim3(KB), 0, s, V, ld, k, h, w, n, rw.partial.p,
                 rw.counter.p, result, bc.vcol, bc.wcol, bc.rcol, bc.hcol);
  HIPCK(hipGetLastError());
}
void launch_update_norm(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, RedWork& rw,
                        double* result, hipStream_t s, const BatchCols& bc) {
  if (k < 1 || k > KMAX) fail(GMG_ERR_INVALID_ARG, "update_norm: bad vector count");
  check_cols(bc);
  GMG_DISPATCH_K(k, k_update_norm, dim3(red_grid(n), bc.nb), dim3(KB), 0, s, V, ld, k, h, w, n, rw.partial.p,
                 rw.counter.p, result, bc.vcol, bc.wcol, bc.rcol, bc.hcol);
  HIPCK(hipGetLastError());
}

__global__ __launch_bounds__(KB) void k_norm2(const double* __restrict__ x, int64_t n, double* partial,
                                              unsigned* counter, double* result, size_t xcol, size_t rcol) {
  x += blockIdx.y * xcol;
  result += blockIdx.y * rcol;
  partial += blockIdx.y * (size_t)KGRID * KMAX;
  counter += blockIdx.y;
  double acc[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    const double v = x[i];
    acc[0] += v * v;
  }
  block_reduce_store<1>(acc, 1, partial, counter, result);
}
void launch_norm2(const double* x, int64_t n, RedWork& rw, double* result, hipStream_t s, int nb, size_t xcol,
                  size_t rcol) {
  if (nb < 1 || nb > KCOLS) fail(GMG_ERR_INVALID_ARG, "norm2: bad column count");
  hipLaunchKernelGGL(k_norm2, dim3(red_grid(n), nb), dim3(KB), 0, s, x, n, rw.partial.p, rw.counter.p, result, xcol,
                     rcol);
  HIPCK(hipGetLastError());
}

// y_c = x_c / sqrt(nrm2[c * rcol]) for the columns c < nb (zero when the
// norm is zero); x_c = x + c * xcol, y_c = y + c * ycol
__global__ void k_normalize_cols(const double* __restrict__ x, size_t xcol, const double* __restrict__ nrm2,
                                 size_t rcol, double* __restrict__ y, size_t ycol, int64_t n) {
  const double nv = nrm2[blockIdx.y * rcol];
  const double hn = sqrt(nv);
  const double a = hn != 0.0 ? 1.0 / hn : 0.0;
  x += blockIdx.y * xcol;
  y += blockIdx.y * ycol;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}
void launch_normalize_cols(const double* x, size_t xcol, const double* nrm2, size_t rcol, double* y, size_t ycol,
                           int64_t n, int nb, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_normalize_cols, dim3((unsigned)g, nb), dim3(256), 0, s, x, xcol, nrm2, rcol, y, ycol, n);
  HIPCK(hipGetLastError());
}

__global__ void k_scale(const double* __restrict__ x, double a, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}
void launch_scale(const double* x, double a, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)g), dim3(256), 0, s, x, a, y, n);
  HIPCK(hipGetLastError());
}

// y = x / sqrt(*nrm2) (zero when the norm is zero), and the basis' Gram
// matrix row `row` (and its mirror column) for the new vector y: block 0
// stores G[row][i] = (V[i] . x) / ||x|| for i < row from the products `dots`
// taken while x was formed (zeros when dots is null: a vector orthogonalised
// by two full passes) and G[row][row] = 1, and copies *nrm2 to nrm2_out when
// that is not null.
__global__ void k_normalize_gram(const double* __restrict__ x, const double* __restrict__ nrm2,
                                 double* __restrict__ y, int64_t n, int row, const double* __restrict__ dots,
                                 double* __restrict__ gram, size_t ldg, double* __restrict__ nrm2_out) {
  const double nv = *nrm2;
  const double hn = sqrt(nv);
  const double a = hn != 0.0 ? 1.0 / hn : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < row; i += blockDim.x) {
      const double gv = dots ? dots[i] * a : 0.0;
      gram[(size_t)row * ldg + i] = gv;
      gram[(size_t)i * ldg + row] = gv;
    }
    if (threadIdx.x == 0) {
      gram[(size_t)row * ldg + row] = 1.0;
      if (nrm2_out) *nrm2_out = nv;
    }
  }
}
void launch_normalize_gram(const double* x, const double* nrm2, double* y, int64_t n, int row, const double* dots,
                           double* gram, size_t ldg, double* nrm2_out, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_normalize_gram, dim3((unsigned)g), dim3(256), 0, s, x, nrm2, y, n, row, dots, gram, ldg,
                     nrm2_out);
  HIPCK(hipGetLastError());
}

template <int K>
__global__ void k_xupdate(double* __restrict__ x, const double* __restrict__ Z, size_t ld, int kc,
                          const double* __restrict__ c, int64_t n, size_t xcol, size_t zcol, size_t ccol) {
  x += blockIdx.y * xcol;
  Z += blockIdx.y * zcol;
  c += blockIdx.y * ccol;
  double ck[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ck[k] = c[k];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v[K];
    double s = x[i];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = Z[k * ld + i];
    ALL_LOADS_ISSUED();
#pragma unroll
    for (int k = 0; k < K; ++k) s += ck[k] * v[k];
    x[i] = s;
  }
}



// Any number of vectors: w <- w - sum_k h[k] V[k] with the coefficients staged
// in LDS; optionally result[0] = ||w_new||^2.  Used when the basis has more
// vectors than one fused pass holds in registers.
__global__ __launch_bounds__(KB) void k_update_many(const double* __restrict__ V, size_t ld, int kc,
                                                    const double* __restrict__ h, double* __restrict__ w,
                                                    int64_t n, int want_norm, double* partial,
                                                    unsigned* counter, double* result) {
  __shared__ double hs[KLDS];
  for (int k = threadIdx.x; k < kc; k += KB) hs[k] = h[k];
  __syncthreads();
  double acc[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    double s = w[i];
    int k = 0;
    for (; k + 16 <= kc; k += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = V[(size_t)(k + u) * ld + i];
      ALL_LOADS_ISSUED();
#pragma unroll
      for (int u = 0; u < 16; ++u) s -= hs[k + u] * v[u];
    }
    for (; k < kc; ++k) s -= hs[k] * V[(size_t)k * ld + i];
    w[i] = s;
    acc[0] += s * s;
  }
  if (want_norm) block_reduce_store<1>(acc, 1, partial, counter, result);
}

void launch_update_many(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, bool want_norm,
                        RedWork& rw, double* result, hipStream_t s) {
  if (k < 1 || k > KLDS) fail(GMG_ERR_INVALID_ARG, "update_many: bad vector count");
  hipLaunchKernelGGL(k_update_many, dim3(red_grid(n)), dim3(KB), 0, s, V, ld, k, h, w, n, want_norm ? 1 : 0,
                     rw.partial.p, rw.counter.p, result);
  HIPCK(hipGetLastError());
}

// ----------------------------------------------------- many-vector passes
// For a basis longer than one register-resident pass: rows are taken in
// chunks of MROWS; thread (r, g) of a block holds rows 2r and 2r + 1 of the
// chunk (one 16-byte load) for the basis vectors g, g + MG, g + 2 MG, ...
// (PER of them, loads all in flight) and keeps their running dot products in
// registers across chunks.  A chunk reads 512 contiguous bytes of each
// vector: shorter segments of many vectors 8 MB apart cost HBM efficiency.
// The block's per-vector sums (over r, in order) go to mpart[block][k]; a
// second kernel adds the blocks in order.  Rows at or past n (the padding up
// to ld, which is a multiple of 64) are loaded but count as zero.
constexpr int MRT = MROWS / 2;    // threads along a chunk's rows

template <int PER>
__device__ __forceinline__ void many_block_sums(const double (&acc)[PER], int kc, double* mpart) {
  // acc[u] of thread (r, g) belongs to vector g + MG u; sum over r in order
  __shared__ double red[MRT][MG + 1];
  const int r = threadIdx.x % MRT, g = threadIdx.x / MRT;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (MG * u >= kc) break;  // the same for every thread of the block
    red[r][g] = acc[u];
    __syncthreads();
    if (threadIdx.x < MG) {
      double t = 0.0;
      for (int q = 0; q < MRT; ++q) t += red[q][threadIdx.x];
      const int k = threadIdx.x + MG * u;
      if (k < kc) mpart[(size_t)blockIdx.x * MSTR + k] = t;
    }
    __syncthreads();
  }
}

// the two rows of thread r in chunk c of V's vector k (zero past n)
__device__ __forceinline__ double2 many_load(const double* __restrict__ V, size_t ld, int k, int64_t i, int64_t n,
                                             bool ok) {
  double2 x = ok ? *reinterpret_cast<const double2*>(V + (size_t)k * ld + i) : make_double2(0.0, 0.0);
  if (i >= n) x.x = 0.0;
  if (i + 1 >= n) x.y = 0.0;
  return x;
}

// h[k] = V[k] . w for k < kc (block partials); the next chunk's loads are
// issued before the current chunk's products
template <int PER>
__global__ __launch_bounds__(MKB) void k_multidot_many(const double* __restrict__ V, size_t ld, int kc,
                                                       const double* __restrict__ w, int64_t n,
                                                       double* __restrict__ mpart) {
  const int r = threadIdx.x % MRT, g = threadIdx.x / MRT;
  double acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = 0.0;
  const int64_t nch = (n + MROWS - 1) / MROWS;
  double2 v[PER], wi;
  auto load = [&](double2 (&x)[PER], double2& xw, int64_t c) {
    const int64_t i = c * MROWS + 2 * r;
    const bool ok = c < nch;
    xw = many_load(w, 0, 0, i, n, ok);
#pragma unroll
    for (int u = 0; u < PER; ++u) x[u] = many_load(V, ld, g + MG * u, i, n, ok && g + MG * u < kc);
  };
  if constexpr (PER <= MPIPE) {
    load(v, wi, blockIdx.x);
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
      double2 vn[PER], wn;
      load(vn, wn, ch + gridDim.x);
      ALL_LOADS_ISSUED();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        acc[u] += v[u].x * wi.x + v[u].y * wi.y;
        v[u] = vn[u];
      }
      wi = wn;
    }
  } else {
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
      load(v, wi, ch);
      ALL_LOADS_ISSUED();
#pragma unroll
      for (int u = 0; u < PER; ++u) acc[u] += v[u].x * wi.x + v[u].y * wi.y;
    }
  }
  many_block_sums<PER>(acc, kc, mpart);
}

// A barrier that orders LDS accesses only: global loads issued before it stay
// in flight (__syncthreads would also wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// w <- w - sum_k h[k] V[k]; block partials of V[k] . w_new, and with
// want_norm of ||w_new||^2 (slot kc).  A chunk's new w needs every vector
// group's partial sum (two barriers per chunk), so the next chunk's basis
// values (and w) are loaded before them.  The grid walks the rows from the
// last chunk down to the first: the preceding multidot pass walked them
// upwards, so the basis rows it read last are still in the 256 MB memory-side
// cache when this pass starts (block b takes chunks nch-1-b, nch-1-b-grid, ...).
template <int PER>
__global__ __launch_bounds__(MKB) void k_update_dot_many(const double* __restrict__ V, size_t ld, int kc,
                                                         const double* __restrict__ h, double* __restrict__ w,
                                                         int64_t n, int want_norm, double* __restrict__ mpart) {
  __shared__ double pr[MROWS][MG + 1];
  __shared__ double wn[MROWS];
  __shared__ double hs[MMAX];
  const int r = threadIdx.x % MRT, g = threadIdx.x / MRT;
  for (int k = threadIdx.x; k < MG * PER; k += MKB) hs[k] = k < kc ? h[k] : 0.0;
  __syncthreads();
  double acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = 0.0;
  const int64_t nch = (n + MROWS - 1) / MROWS;
  double2 v[PER];
  // step c of the walk is chunk nch - 1 - c
  auto load = [&](double2 (&x)[PER], int64_t c) {
    const int64_t i = (nch - 1 - c) * MROWS + 2 * r;
    const bool ok = c < nch;
#pragma unroll
    for (int u = 0; u < PER; ++u) x[u] = many_load(V, ld, g + MG * u, i, n, ok && g + MG * u < kc);
  };
  // threads 0..MROWS-1 also hold w of their row of the chunk (loaded one
  // chunk ahead, like the basis values)
  auto load_w = [&](int64_t c) {
    const int64_t ii = (nch - 1 - c) * MROWS + threadIdx.x;
    return (threadIdx.x < MROWS && c < nch && ii < n) ? w[ii] : 0.0;
  };
  double wc = load_w(blockIdx.x);
  double nacc = 0.0;  // threads 0..MROWS-1 (wave 0): squares of their rows of w_new
  if constexpr (PER <= MPIPE) load(v, blockIdx.x);
  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const int64_t ch = nch - 1 - c;
    double2 vn[PER];
    const double wnext = load_w(c + gridDim.x);
    if constexpr (PER <= MPIPE) load(vn, c + gridDim.x);
    else load(v, c);
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const double hk = hs[g + MG * u];
      p0 += hk * v[u].x;
      p1 += hk * v[u].y;
    }
    pr[2 * r][g] = p0;
    pr[2 * r + 1][g] = p1;
    lds_barrier();
    if (threadIdx.x < MROWS) {
      const int64_t ii = ch * MROWS + threadIdx.x;
      double t = 0.0;
      if (ii < n) {
        t = wc;
        for (int q = 0; q < MG; ++q) t -= pr[threadIdx.x][q];
        w[ii] = t;
      }
      wn[threadIdx.x] = t;
      nacc += t * t;
    }
    wc = wnext;
    lds_barrier();
    const double w0 = wn[2 * r], w1 = wn[2 * r + 1];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      acc[u] += v[u].x * w0 + v[u].y * w1;
      if constexpr (PER <= MPIPE) v[u] = vn[u];
    }
  }
  __syncthreads();
  many_block_sums<PER>(acc, kc, mpart);
  static_assert(MROWS == 64, "the norm is reduced within wave 0");
  if (want_norm && threadIdx.x < MROWS) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nacc += __shfl_down(nacc, off, 64);
    if (threadIdx.x == 0) mpart[(size_t)blockIdx.x * MSTR + kc] = nacc;
  }
}

// result[k] = sum over blocks b (in order) of mpart[b][k]; 8 vectors per
// block, MPARTS thread groups each adding every MPARTS-th block, then the
// groups in order
__global__ __launch_bounds__(KB) void k_colsum(const double* __restrict__ mpart, int nb, int kc,
                                               double* __restrict__ result) {
  constexpr int NC = KB / MPARTS;
  __shared__ double sh[MPARTS][NC];
  const int c = threadIdx.x % NC, part = threadIdx.x / NC;
  const int k = blockIdx.x * NC + c;
  double s = 0.0;
  if (k < kc) {
    constexpr int IN = MGRID / MPARTS;
    double v[IN];
#pragma unroll
    for (int u = 0; u < IN; ++u) {
      const int b = part + u * MPARTS;
      v[u] = b < nb ? mpart[(size_t)b * MSTR + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < IN; ++u) s += v[u];
  }
  sh[part][c] = s;
  __syncthreads();
  if (threadIdx.x < NC && k < kc) {
    double t = 0.0;
    for (int q = 0; q < MPARTS; ++q) t += sh[q][threadIdx.x];
    result[k] = t;
  }
}

static unsigned many_grid(int64_t n) {
  int64_t g = (n + MROWS - 1) / MROWS;
  if (g > MGRID) g = MGRID;
  if (g < 1) g = 1;
  return (unsigned)g;
}

#define GMG_MANY(KERNEL, kc, ...)                                                  \
  do {                                                                             \
    const int per_ = (kc + MG - 1) / MG;                                           \
    if (per_ <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                     \
    else if (per_ <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);              \
    else hipLaunchKernelGGL(KERNEL<24>, __VA_ARGS__);                              \
  } while (0)

static_assert(MMAX <= 24 * MG, "the widest many-vector instance holds 24 vectors per group");
int many_max() { return MMAX; }

void launch_multidot_many(const double* V, size_t ld, int k, const double* w, int64_t n, RedWork& rw, double* result,
                          hipStream_t s) {
  if (k < 1 || k > MMAX) fail(GMG_ERR_INVALID_ARG, "multidot_many: bad vector count");
  const unsigned nb = many_grid(n);
  GMG_MANY(k_multidot_many, k, dim3(nb), dim3(MKB), 0, s, V, ld, k, w, n, rw.mpart.p);
  hipLaunchKernelGGL(k_colsum, dim3((k + KB / MPARTS - 1) / (KB / MPARTS)), dim3(KB), 0, s, rw.mpart.p, (int)nb, k,
                     result);
  HIPCK(hipGetLastError());
}

void launch_update_dot_many(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, bool want_norm,
                            RedWork& rw, double* result, hipStream_t s) {
  if (k < 1 || k > MMAX) fail(GMG_ERR_INVALID_ARG, "update_dot_many: bad vector count");
  const unsigned nb = many_grid(n);
  const int wn = want_norm ? 1 : 0;
  GMG_MANY(k_update_dot_many, k, dim3(nb), dim3(MKB), 0, s, V, ld, k, h, w, n, wn, rw.mpart.p);
  hipLaunchKernelGGL(k_colsum, dim3((k + wn + KB / MPARTS - 1) / (KB / MPARTS)), dim3(KB), 0, s, rw.mpart.p, (int)nb,
                     k + wn, result);
  HIPCK(hipGetLastError());
}

// Gram-corrected coefficients of one projection: with G = V^T V (unit
// diagonal taken as exact), c = h + d, d_i = -sum_{l != i} G[i][l] h[l],
// i.e. c = (2I - G) h, the first-order form of G^{-1} h: the same as a second
// classical Gram-Schmidt pass, V^T (w - V h) = h - G h, without reading V
// again.  One wave per coefficient, lanes over l, added in a fixed order.
__global__ __launch_bounds__(64) void k_gram_coef(int kc, const double* __restrict__ h,
                                                  const double* __restrict__ gram, size_t ldg,
                                                  double* __restrict__ d, double* __restrict__ c) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const double* gi = gram + (size_t)i * ldg;
  double s = 0.0;
  for (int l = lane; l < kc; l += 64)
    if (l != i) s += gi[l] * h[l];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    d[i] = -s;
    c[i] = h[i] + (-s);
  }
}
void launch_gram_coef(int kc, const double* h, const double* gram, size_t ldg, double* d, double* c,
                      hipStream_t s) {
  if (kc < 1) return;
  hipLaunchKernelGGL(k_gram_coef, dim3(kc), dim3(64), 0, s, kc, h, gram, ldg, d, c);
  HIPCK(hipGetLastError());
}
#undef GMG_MANY


__global__ __launch_bounds__(KB) void k_xupdate_many(double* __restrict__ x, const double* __restrict__ Z, size_t ld,
                                                     int kc, const double* __restrict__ c, int64_t n) {
  __shared__ double cs[KLDS];
  for (int k = threadIdx.x; k < kc; k += KB) cs[k] = c[k];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    double s = x[i];
    int k = 0;
    for (; k + 16 <= kc; k += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = Z[(size_t)(k + u) * ld + i];
      ALL_LOADS_ISSUED();
#pragma unroll
      for (int u = 0; u < 16; ++u) s += cs[k + u] * v[u];
    }
    for (; k < kc; ++k) s += cs[k] * Z[(size_t)k * ld + i];
    x[i] = s;
  }
}

__global__ void k_get_col(const double* __restrict__ X, int nrhs, int col, double* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = X[i * nrhs + col];
}
__global__ void k_set_col(double* __restrict__ X, int nrhs, int col, const double* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i * nrhs + col] = x[i];
}
void launch_get_col(const double* X, int nrhs, int col, double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_get_col, dim3((unsigned)g), dim3(256), 0, s, X, nrhs, col, x, n);
  HIPCK(hipGetLastError());
}
void launch_set_col(double* X, int nrhs, int col, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_set_col, dim3((unsigned)g), dim3(256), 0, s, X, nrhs, col, x, n);
  HIPCK(hipGetLastError());
}

void launch_xupdate(double* x, const double* Z, size_t ld, int k, const double* c, int64_t n, hipStream_t s, int nb,
                    size_t xcol, size_t zcol, size_t ccol) {
  if (n <= 0 || k <= 0) return;
  if (nb < 1 || nb > KCOLS || (nb > 1 && k > KMAX)) fail(GMG_ERR_INVALID_ARG, "xupdate: bad column count");
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (nb > 1 && g > 1024) g = 1024;
  if (k <= KMAX) {
    GMG_DISPATCH_K(k, k_xupdate, dim3((unsigned)g, nb), dim3(256), 0, s, x, Z, ld, k, c, n, xcol, zcol, ccol);
  } else {
    if (k > KLDS) fail(GMG_ERR_INVALID_ARG, "xupdate: bad vector count");
    hipLaunchKernelGGL(k_xupdate_many, dim3((unsigned)g), dim3(KB), 0, s, x, Z, ld, k, c, n);
  }
  HIPCK(hipGetLastError());
}

}  // namespace gmg
