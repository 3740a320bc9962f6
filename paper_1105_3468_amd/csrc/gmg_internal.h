// Internal declarations of the MI355X two-grid matching-AMG library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gmg.h"

namespace gmg {

// ---------------------------------------------------------------- errors
struct Error {
  gmg_status code;
  std::string msg;
};
[[noreturn]] void fail(gmg_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCK(x) ::gmg::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------- memory
// Device memory comes from a per-device cache of freed blocks (pool.cpp):
// pool_alloc returns nullptr on failure.  While a PoolStream is alive on the
// calling thread, blocks freed by it are tagged with its stream and reused on
// that stream without waiting; without one they go back to the runtime.
// pool_idle(s): the caller has synchronised s, so blocks freed on s may be
// reused on any stream.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
void pool_idle(hipStream_t s);
class PoolStream {
 public:
  explicit PoolStream(hipStream_t s);
  ~PoolStream();
  PoolStream(const PoolStream&) = delete;
  PoolStream& operator=(const PoolStream&) = delete;

 private:
  bool had_;
  hipStream_t prev_;
};

// Owning device buffer (library-allocated).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    p = static_cast<T*>(pool_alloc(count * sizeof(T)));
    if (!p) {
      n = 0;
      fail(GMG_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
  }
  void release() {
    if (p) pool_free(p);
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
};

template <class T>
void h2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) HIPCK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
void d2h(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) HIPCK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
}
template <class T>
void d2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) HIPCK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

// Device CSR matrix owned by the library.
struct DCsr {
  int n = 0, m = 0;          // rows, columns
  int64_t nnz = 0;
  DBuf<int> rp, ci;
  DBuf<double> v;
  DBuf<float> v32;
};

// Host CSR (for analysis steps).
struct HCsr {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
};

// A narrow triangular factor prepared for the single-CU sweep: entries e in
// schedule order (level by level, lptr[l] .. lptr[l+1]), entry e is row
// rows[e]; its `width` operands are LDS ring slots wslot[e*width + k] with
// values wval[...] (slot CU_RING*1024 is a zero used as padding); dinv_e[e]
// is the reciprocal diagonal of row rows[e] when the factor stores one.
struct CuSweep {
  int n = 0, levels = 0, width = 0;
  bool has_diag = false;
  DBuf<int> lptr, rows, wslot;
  DBuf<double> wval, dinv_e;
  DBuf<float> wval32, dinv_e32;
};

// A triangular factor prepared for the synchronisation-free sweep: row rows[e]
// (entries e in schedule order: by dependency level, ascending row inside a
// level) has dependency entries dcol[dp[e] .. dp[e+1]) with values dval.
// chunk[3c .. 3c+2] = (first entry, rows, log2 lanes per row) of wave chunk c;
// a chunk holds rows of a single level.  out[r] = (rhs[r] - sum dval *
// out[dcol]) * dinv[r] (dinv only for factors with a stored diagonal).
struct Sweep {
  int n = 0;                 // rows of the factor
  int nchunks = 0;
  int levels = 0;
  int64_t nnz = 0;           // dependency entries
  DBuf<int> chunk, rows, dp, dcol;
  DBuf<double> dval, dinv;
  DBuf<float> dval32, dinv32;
  DBuf<unsigned> ticket;     // dynamic chunk counter
  unsigned ticket_base = 0;  // host copy of the counter value at the next launch
  bool has_diag = false;
  int waves = 0;             // resident waves (a few dependency levels of look-ahead)
  // consecutive level ranges, one launch each: chunks [seg_c0[g], seg_c1[g])
  // (rows = entries [seg_e0[g], seg_e1[g])) on one workgroup with the
  // range's results in LDS (seg_wg[g] != 0) or on the whole device.  For
  // entries of one-workgroup ranges, dslot[q] is the LDS slot of dependency
  // dcol[q] when it lies in the same range, else -1 - dcol[q].
  std::vector<int> seg_c0, seg_c1, seg_e0, seg_e1;
  std::vector<char> seg_wg;
  std::vector<int> lvl_c0;   // first chunk of each dependency level (levels + 1 entries)
  DBuf<int> dslot;
  std::unique_ptr<CuSweep> cu;  // single-CU form, for narrow factors (null otherwise)
};

// Wavefront sweeps of factors with 2D- or 3D-grid structure (k_wave.hip).
// 2D (nz == 0): grid of nx columns and ny rows, W waves of 64 grid rows,
// S = nx + 63 steps per wave (rounded up).  3D: nx x ny x nz cells, W = TY * TZ
// tiles of 8 x 8 grid lines (TY = ceil(ny / 8)), S = nx + 14 steps
// (rounded up).  total = W * S * 64 positions (the lower layout; an upper
// factor uses it backwards).
struct WaveGrid {
  int nx = 0, ny = 0, W = 0, S = 0;
  int nz = 0, TY = 0;
  int64_t total = 0;
};
// One factor in that layout.  2D: coef holds (neighbour below, left
// neighbour) coefficient pairs per position, zero where absent or outside the
// grid, and dinv the reciprocal diagonal per position when the factor stores
// one.  3D: coef holds (z, y, x neighbour, reciprocal diagonal) quads.
struct WaveSweep {
  bool has_diag = false;
  DBuf<double> coef, dinv;
  DBuf<float> coef32, dinv32;
};
// z (natural order, FP64 if z_f64) -> lower sweep -> upper sweep -> t
// (natural order); zs, ys, ts are layout-ordered work vectors, ys and ts
// all-sentinel on entry and left so.
template <class T>
void launch_wave_pair(const WaveGrid& g, const WaveSweep& lo, const WaveSweep& up, const void* z, bool z_f64, T* zs,
                      T* ys, T* ts, T* t, int* abort_flag, hipStream_t s, int nb = 1, size_t ldz = 0,
                      size_t ldt = 0);

// A triangular factor solved over the nested-dissection tree (k_tree.hip):
// tasks in tree order, 8 ints each (kind 0: helper for rows [r0, r1) of a
// node, kind 1: the node's own solve; lo, s = the node's rows; node index
// into boff; has_ext; log2 lanes per row for helpers); erp/ecol/eval: per row,
// the entries outside the row's node; blk: each node's diagonal block, dense
// s x s column-major at boff[node] (zeros where the factor has none); dinv:
// reciprocal diagonal per row (factors with a stored diagonal).
constexpr int kTreeMaxRows = 2048;  // rows of one node (its values are staged in LDS)
constexpr int kDenseMaxCoarse = 8192;  // largest A_c of the dense exact coarse solve (512 MiB in FP64)
// A triangular factor laid out for the tree solve: per task 8 ints (helper
// or node slice), outside entries as CSR over rows (erp, ecol, eval), and per
// node the inverse of its diagonal block, dense column-major at boff[node]
// (zeros in the other triangle); ncount[node] counts the node's slices
// arriving in a solve (zero between solves).
struct TreeSolve {
  bool lower = true, has_diag = false;
  int ntasks = 0, max_rows = 0, heights = 0;
  DBuf<int> task, erp, ecol, ncount;
  DBuf<int64_t> boff;
  DBuf<double> eval, inv;
  DBuf<float> eval32, inv32;
};
template <class T>
void launch_tree(const TreeSolve& ts, const void* rhs, bool rhs_is_f64, T* out, T* reset_rhs, T* ext,
                 int* abort_flag, hipStream_t s, int nb = 1, size_t ld = 0, int* ncount = nullptr);
// Setup: inverses of the diagonal blocks blk (same layout as inv) into inv,
// one workgroup per task (8 ints: lo, s, c0, node, log2 W; a chunk of W
// columns of one node), with `lds` bytes of LDS (tree_inv_lds of each task,
// at most kTreeInvLds).
constexpr size_t kTreeInvLds = 128 * 1024;
// Setup: dense diagonal blocks (zeroed beforehand) and outside-entry lists of
// a factor whose row r holds entries [rp[r] + skip, rp[r+1]).
void launch_tree_fill(int n, const int* rp, const int* ci, const double* v, int skip, const int* node_of,
                      const int* nlo, const int* nsz, const int64_t* boff, const int* erp, double* blk, int* ecol,
                      double* eval, hipStream_t s);
size_t tree_inv_lds(int rows, int lgW);
int tree_inv_width(int rows);
void launch_tree_invert(const TreeSolve& ts, const int* itask, int ntask, size_t lds, const double* blk,
                        const double* dinv, double* inv, hipStream_t s);

// Per-kernel-class profiling with events.
enum ProfClass {
  PC_SPMV = 0, PC_SWEEP_FINE, PC_SWEEP_COARSE, PC_RESID_RESTRICT, PC_PROLONG,
  PC_ORTHO, PC_VECTOR, PC_COUNT
};

struct Solver;

// ---------------------------------------------------------------- kernels
// Sparse kernels (k_sparse.hip)
void launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s);
void launch_fill_f64_bits(double* p, uint64_t bits, size_t n, hipStream_t s);
void launch_fill_f32_bits(float* p, uint32_t bits, size_t n, hipStream_t s);
void launch_validate(int n, const int* rp, const int* ci, const double* v, int* flags,
                     hipStream_t s);
void launch_cast_f32(const double* x, float* y, size_t n, hipStream_t s);
// dense exact coarse solve (k_dense.hip): A (np x np, row-major, np a multiple
// of 64 >= nc) <- blockdiag(A_c, I)^{-1}; *bad set to 1 on a zero or
// non-finite pivot
void launch_dense_inverse(int nc, int np, const int* rp, const int* ci, const double* v, double* A, int* bad,
                          hipStream_t s);
template <class T>
void launch_dense_gemv(int n, int np, const T* M, const T* r, T* e, hipStream_t s);
// MT = M^T (leading n x n block, row stride np)
void launch_dense_transpose(int n, int np, const double* M, double* MT, hipStream_t s);
// CSR SpMV y = A x; T = value/vector type.  cap: products of a 256-row tile
// staged in LDS (2048 or 4096; spmv_cap picks it from the largest tile, and
// tiles beyond it are computed from global memory)
int spmv_cap(int64_t max_tile_nnz);
template <class T>
void launch_spmv(int n, const int* rp, const int* ci, const T* v, const T* x, T* y,
                 hipStream_t s, int cap = 4096);
// r = b - A x  (r may alias nothing); FP64 only
void launch_residual(int n, const int* rp, const int* ci, const double* v, const double* x,
                     const double* b, double* r, hipStream_t s, int cap = 4096);
// Fine residual of the smoothed iterate: r[k] = z[k] - (A t)[k]  (Tz = input type)
template <class T>
void launch_resid_fine(int n, const int* rp, const int* ci, const T* v, const T* t,
                       const double* z, T* r, hipStream_t s, int cap = 4096);
// rc[I] = sum_{k in G_I} r[k]; also writes the sentinel into reset[I]
template <class T>
void launch_restrict(int nc, const int* aptr, const int* amem, const T* r, T* rc, T* reset,
                     uint64_t sentinel_bits, hipStream_t s);
// q[k] = t[k] + ec[agg[k]] (q in double); t[k] <- sentinel when reset_t
template <class T>
void launch_prolong(int n, const int* agg, T* t, const T* ec, double* q, uint64_t sentinel_bits,
                    hipStream_t s, bool reset_t = true);
// Adjoint helpers
void launch_restrict_plain(int nc, const int* aptr, const int* amem, const double* z,
                           double* bc, double* reset, uint64_t sentinel_bits, hipStream_t s);
// s[k] = z[k] - sum_l AT[k,l] ec[agg[l]]
void launch_resid_adj(int n, const int* rp, const int* ci, const double* v, const int* agg,
                      const double* ec, const double* z, double* out, hipStream_t s);
// Transpose a device CSR (n rows, m cols) into T (m rows, n cols); columns ascending.
void transpose_csr(int n, int m, int64_t nnz, const int* rp, const int* ci, const double* v,
                   DBuf<int>& trp, DBuf<int>& tci, DBuf<double>* tv, DBuf<int>* tsrc,
                   hipStream_t s);
void launch_gather_f64(const double* src, const int* idx, double* dst, int64_t n, hipStream_t s);
// zp[k] = z[perm[k]]; and t[perm[k]] = tp[k] with tp reset to the sentinel
template <class T>
void launch_perm_gather(int n, const int* perm, const double* z, T* zp, hipStream_t s);
template <class T>
void launch_perm_scatter(int n, const int* perm, T* tp, T* t, hipStream_t s);
void launch_exclusive_scan_int(const int* in, int* out, int n, hipStream_t s, DBuf<int>& tmp);
void launch_exclusive_scan_int_ws(const int* in, int* out, int n, int* bsum, hipStream_t s);
constexpr int SCAN_BLOCK = 1024;  // elements per block of the exclusive scan
// message returned by gmg_last_error() on this thread
void set_error_message(const std::string& msg);

// Triangular sweeps (k_sweep.hip)
// One launch per dependency level (no polling: a level reads earlier levels'
// results as final values); for factors with a few wide levels.
constexpr int kLevelLaunchMax = 16;
template <class T>
void launch_sweep_levels(Sweep& sw, const T* dval, const T* dinv, const void* rhs, bool rhs_is_f64, T* out,
                         T* reset_rhs, hipStream_t s);
template <class T>
void launch_sweep(Sweep& sw, const T* dval, const T* dinv, const void* rhs, bool rhs_is_f64,
                  T* out, T* reset_rhs, int waves, bool whole, int* abort_flag, hipStream_t s);
// rows of a one-workgroup level range (its FP64 results fill 128 KiB of LDS)
constexpr int kSweepLdsRows = 16384;
template <class T>
void launch_cu_sweep(CuSweep& cs, const T* wval, const T* dinv_e, const void* rhs, bool rhs_is_f64, T* out,
                     T* reset_rhs, T* rhs_s, T* out_s, hipStream_t s);
// ILU(0) of a matrix with the 2D-grid structure (offsets -/+1 within grid
// rows and -/+nx, nx >= 3, ny <= 4096): one launch over the anti-diagonals,
// bitwise equal to the level-scheduled kernel
bool ilu0_grid_fits(int nx, int ny);
void launch_ilu0_grid(int n, int nx, const int* rp, const int* ci, const int* dpos, double* a, int* bad,
                      hipStream_t s);
void launch_ilu0_level(const int* rows, int count, const int* rp, const int* ci, const int* dpos,
                       double* a, int* bad, hipStream_t s);
// yout[i] = (b[i] - sum_{j != i} F_ij yin[j]) * (dinv ? dinv[i] : 1)
void launch_jacobi(int n, const int* rp, const int* ci, const double* v, const double* dinv, const double* b,
                   const double* yin, double* yout, hipStream_t s);

// Krylov kernels (k_krylov.hip)
struct RedWork {  // scratch for deterministic two-level reductions
  DBuf<double> partial;
  DBuf<double> mpart;    // block partials of the many-vector passes
  DBuf<unsigned> counter;
  DBuf<double> result;   // two coefficient blocks of up to 2048 values + norms
  int blocks = 0;
};
void red_init(RedWork& rw, hipStream_t s);
void red_reset(RedWork& rw, hipStream_t s);
// Independent recurrences batched in one launch of the k <= 32 Krylov
// kernels: column c (c < nb) works on V + c * vcol, w + c * wcol, h + c * hcol
// and writes result + c * rcol.
constexpr int KCOLS = 16;
struct BatchCols {
  int nb = 1;
  size_t vcol = 0, wcol = 0, rcol = 0, hcol = 0;
};
// result[0..k) = V[0..k)^T w   (V rows with stride ld)
void launch_multidot(const double* V, size_t ld, int k, const double* w, int64_t n,
                     RedWork& rw, double* result, hipStream_t s, const BatchCols& bc = BatchCols());
// w -= V[0..k)^T h  (h device), then result[0..k) = V^T w_new
void launch_update_dot(const double* V, size_t ld, int k, const double* h, double* w, int64_t n,
                       RedWork& rw, double* result, hipStream_t s, const BatchCols& bc = BatchCols());
// w -= V^T h, then result[0] = ||w||^2
void launch_update_norm(const double* V, size_t ld, int k, const double* h, double* w, int64_t n,
                        RedWork& rw, double* result, hipStream_t s, const BatchCols& bc = BatchCols());
// any k (<= 2048): w -= V^T h (h device); if want_norm, result[0] = ||w_new||^2
// Many-vector passes (up to many_max() vectors): result[0..k) = V^T w, and
// w <- w - V h with result[0..k) = V^T w_new (and result[k] = ||w_new||^2
// when want_norm), each reading V once.
int many_max();
void launch_multidot_many(const double* V, size_t ld, int k, const double* w, int64_t n, RedWork& rw, double* result,
                          hipStream_t s);
void launch_update_dot_many(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, bool want_norm,
                            RedWork& rw, double* result, hipStream_t s);
// c = (2I - G) h and d = c - h for the basis' Gram matrix G (row-major, ldg;
// unit diagonal assumed): the coefficients of a projection corrected for the
// basis' loss of orthogonality, as a second Gram-Schmidt pass would give
void launch_gram_coef(int kc, const double* h, const double* gram, size_t ldg, double* d, double* c,
                      hipStream_t s);
// y = x / sqrt(*nrm2) (zero when *nrm2 is zero), and the Gram row of y:
// G[row][i] = G[i][row] = dots[i] / sqrt(*nrm2) (i < row; zeros if dots is
// null), G[row][row] = 1; *nrm2_out = *nrm2 when nrm2_out is not null
void launch_normalize_gram(const double* x, const double* nrm2, double* y, int64_t n, int row, const double* dots,
                           double* gram, size_t ldg, double* nrm2_out, hipStream_t s);
void launch_update_many(const double* V, size_t ld, int k, const double* h, double* w, int64_t n, bool want_norm,
                        RedWork& rw, double* result, hipStream_t s);
// result[0] = ||x||^2
void launch_norm2(const double* x, int64_t n, RedWork& rw, double* result, hipStream_t s, int nb = 1,
                  size_t xcol = 0, size_t rcol = 0);
// y_c = x_c / sqrt(nrm2[c * rcol]) for columns c < nb (x_c = x + c * xcol, ...)
void launch_normalize_cols(const double* x, size_t xcol, const double* nrm2, size_t rcol, double* y, size_t ycol,
                           int64_t n, int nb, hipStream_t s);
// y = alpha * x
void launch_scale(const double* x, double alpha, double* y, int64_t n, hipStream_t s);
// x += sum_i c[i] Z[i]  (c device)
void launch_xupdate(double* x, const double* Z, size_t ld, int k, const double* c, int64_t n,
                    hipStream_t s, int nb = 1, size_t xcol = 0, size_t zcol = 0, size_t ccol = 0);
// strided column gather/scatter for multi-RHS
void launch_get_col(const double* X, int nrhs, int col, double* x, int64_t n, hipStream_t s);
void launch_set_col(double* X, int nrhs, int col, const double* x, int64_t n, hipStream_t s);

// Multi-right-hand-side kernels (k_batch.hip): nb <= BATCH_MAX columns per
// launch, column c of a batch at base + c * ld.
constexpr int BATCH_MAX = 16;
template <class T>
void launch_spmm(int n, const int* rp, const int* ci, const T* v, const T* x, size_t ldx, T* y, size_t ldy, int nb,
                 hipStream_t s);
// r_c = b_c - A x_c
void launch_residual_cols(int n, const int* rp, const int* ci, const double* v, const double* x, size_t ldx,
                          const double* b, size_t ldb, double* r, size_t ldr, int nb, hipStream_t s);
// out_c = z_c - A^T P ec_c (rp/ci/v: A^T as CSR)
void launch_resid_adj_cols(int n, const int* rp, const int* ci, const double* v, const int* agg, const double* ec,
                           size_t ldc, const double* z, size_t ldz, double* out, size_t ldo, int nb, hipStream_t s);
// r_c = z_c - A t_c (t and r in precision T, z FP64)
template <class T>
void launch_resid_fine_cols(int n, const int* rp, const int* ci, const T* v, const T* t, size_t ldt, const double* z,
                            size_t ldz, T* r, size_t ldr, int nb, hipStream_t s);
// rc_c = P^T r_c in precision T; reset_c <- sentinel (reset may be null)
template <class T>
void launch_restrict_cols_t(int nc, const int* aptr, const int* amem, const T* r, size_t ldr, T* rc, T* reset,
                            size_t ldc, int nb, hipStream_t s);
// rc_c = P^T z_c; reset_c <- sentinel (reset may be null)
void launch_restrict_cols(int nc, const int* aptr, const int* amem, const double* z, size_t ldz, double* rc,
                          double* reset, size_t ldc, int nb, hipStream_t s);
// q_c = t_c + P ec_c (widened to FP64); t_c <- sentinel
template <class T>
void launch_prolong_cols(int n, const int* agg, T* t, size_t ldt, const T* ec, size_t ldc, double* q, size_t ldq,
                         int nb, hipStream_t s);
// out_c[i] = X[i * nrhs + c0 + c] (c < nb), and the reverse
void launch_cols_from_rows(const double* X, int nrhs, int c0, double* out, size_t ld, int64_t n, int nb,
                           hipStream_t s);
void launch_rows_from_cols(double* X, int nrhs, int c0, const double* in, size_t ld, int64_t n, int nb,
                           hipStream_t s);

// Setup kernels (k_setup.hip)
void build_graph(int n, const int* rp, const int* ci, const double* v, const int* trp,
                 const int* tci, const double* tv, DBuf<int>& grp, DBuf<int>& gci,
                 DBuf<double>& gw, hipStream_t s);
// Multi-pass handshake matching; returns N_c, fills agg (device int[n]).
int aggregate(int n, const DBuf<int>& grp, const DBuf<int>& gci, const DBuf<double>& gw,
              double cf, int max_passes, int qbits, uint64_t seed, DBuf<int>& agg,
              int* passes, int* rounds, hipStream_t s);
// Member lists (P^T as CSR) of agg.
void build_members(int n, int nc, const int* agg, DBuf<int>& aptr, DBuf<int>& amem,
                   hipStream_t s);
// agg[k] <- rank[agg[k]]
void relabel(int n, int* agg, const int* rank, hipStream_t s);
// Galerkin A_c = P^T A P with sums in the fine CSR order.
void galerkin(int n, int nc, const int* rp, const int* ci, const double* v, const int* agg,
              const int* aptr, const int* amem, DCsr& Ac, hipStream_t s);

// Host analysis (host_analysis.cpp)
// Level schedule of a triangular dependency structure given as per-row
// dependency lists (host CSR): lower = dependencies have smaller index.
// level_ptr[l] is the first schedule position of level l (levels padded to 64).
void make_schedule(const std::vector<int>& dep_rp, const std::vector<int>& dep_ci, bool lower,
                   std::vector<int>& sched, std::vector<int>& level_ptr, int* levels);
// Nested-dissection numbering (position -> vertex) of a symmetric graph.  A
// node of the dissection tree owns the positions [lo, hi) (a leaf's subgraph,
// or the separator of its two children; empty for a split into components)
// and is numbered after all of its descendants; height 0 for leaves.
struct NdNode {
  int lo, hi, parent, height;
};
std::vector<int> nd_numbering(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                              std::vector<NdNode>* tree = nullptr);
// Colour-class numbering (position -> vertex) of a symmetric graph: greedy
// colouring in natural order (smallest colour unused by earlier neighbours),
// vertices listed by colour, ascending within a colour.
std::vector<int> color_numbering(int n, const std::vector<int>& rp, const std::vector<int>& ci);
// Row-wise ILUT(tau) without pivoting on a host CSR; L strictly lower,
// U with the diagonal first.  Returns GMG_OK / GMG_ERR_ZERO_PIVOT / NONFINITE.
// With the nested-dissection tree of A's numbering, the tree's nodes are
// factored in parallel (same result).
gmg_status host_ilut(const HCsr& A, double tau, HCsr& L, HCsr& U, const std::vector<NdNode>* tree = nullptr);
// Sparse approximate inverse of A with A's pattern (each column the
// least-squares minimiser of ||A m - e_j|| over its column's pattern), on
// host threads.  GMG_OK / GMG_ERR_ZERO_PIVOT (rank-deficient column block) /
// GMG_ERR_NONFINITE.
gmg_status host_spai(const HCsr& A, HCsr& M);
// host worker threads: GMG_THREADS, else OMP_NUM_THREADS, else the hardware's
// (at most 64)
int host_threads();

}  // namespace gmg
