// C ABI, setup pipeline and the FGMRES driver of the two-grid matching-AMG
// solver.  The host only sequences kernels and reads back a handful of
// scalars per Krylov step; every vector operation runs on the GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <exception>
#include <thread>
#include <vector>

#include "gmg_internal.h"

namespace gmg {

static thread_local std::string g_last_error;

void set_error_message(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(gmg_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  gmg_status code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? GMG_ERR_OOM : GMG_ERR_HIP;
  fail(code, std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")");
}

constexpr uint64_t kSent64 = 0x7FF8DEADBEEFF00DULL;
constexpr uint32_t kSent32 = 0x7FC0FEEDu;
constexpr int kMaxRestart = 2048;   // longest Krylov basis (vectors)
constexpr int kPinCol = 2 * kMaxRestart + 8;  // doubles per pinned block (scalars, or h1, h2, ||w||^2)
constexpr int kFused = 32;          // basis size handled by the fused CGS2 kernels

static const char* kProfNames[PC_COUNT] = {"spmv", "sweep_fine", "sweep_coarse", "resid_restrict",
                                           "prolong", "ortho", "vector"};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};

// Workspace of the multi-right-hand-side solve: up to BATCH_MAX columns,
// column-major, fine vectors ld apart, coarse vectors ldc apart, Krylov bases
// of m steps (step j of column c at V + (j * cap + c) * ld).
struct BatchWork {
  int cap = 0, m = 0;
  size_t ld = 0, ldc = 0;
  bool f32 = false, adj = false;
  DBuf<double> t, rc, yc, ec, wz, wy, wt, text;                    // FP64 cycle
  DBuf<float> t32, rc32, yc32, ec32, wz32, wy32, wt32, text32;     // FP32 cycle
  DBuf<int> ncLc, ncUc, ncUct, ncLct;                              // tree node counters per column
  DBuf<double> abc, auc, aec, as, at;                              // adjoint cycle
  DBuf<double> r;                                                  // fine residuals before the restriction
  DBuf<float> r32;
  DBuf<double> V, Z, w, x, b, coef;                                // Krylov
};

struct Solver {
  hipStream_t s = nullptr;
  gmg_options opt{};
  int n = 0;
  int64_t nnz = 0;
  DCsr A, AT;
  DBuf<int> agg, aptr, amem;
  int nc = 0, passes = 0, rounds = 0;
  DCsr Ac;
  DBuf<double> ilu, u0dinv;    // ILU(0) values (A's pattern), U0's reciprocal diagonal
  DBuf<int> dpos, at_src;      // diagonal positions; A^T entry -> A entry
  bool adj_ready = false;      // transposed factors built (on first adjoint use)
  HCsr hLc, hUc;
  Sweep L0, U0, Lc, Uc;        // forward factors
  Sweep U0t, L0t, Uct, Lct;    // transposed factors (adjoint)
  DCsr dLc, dUc;               // coarse factors as CSR (Jacobi mode)
  DCsr dLcT, dUcT;             // their transposes (adjoint Jacobi sweeps)
  DCsr dMcT;                   // transposed sparse approximate inverse (adjoint)
  DBuf<double> cinvT;          // transposed dense inverse (adjoint)
  HCsr hMc;                    // sparse approximate inverse of A_c (coarse_mode 2)
  DCsr dMc;
  DBuf<double> cinv;           // dense A_c^{-1}, padded row-major (coarse_mode 3)
  DBuf<float> cinv32;
  DBuf<int> cbad;
  int cnp = 0;                 // its padded size
  DBuf<double> ucdinv, jzero, jtmp;
  // forward V-cycle work vectors
  DBuf<double> y, t, r, rc, yc, ec;
  DBuf<float> y32, t32, r32, rc32, yc32, ec32;
  // adjoint V-cycle work vectors
  DBuf<double> abc, auc, aec, as, aw, at;
  // schedule-order staging of the single-CU sweeps
  DBuf<double> cu_rhs, cu_out;
  DBuf<float> cu_rhs32, cu_out32;
  // coarse factors solved over the nested-dissection tree
  std::vector<NdNode> nd_tree;
  bool tree = false, tree_adj = false;
  TreeSolve tLc, tUc, tUct, tLct;
  DBuf<double> text;
  DBuf<float> text32;
  // wavefront form of the fine factors (2D-grid structure)
  bool wave = false;
  WaveGrid wg;
  WaveSweep wL0, wU0, wU0t, wL0t;
  DBuf<double> wz, wy, wt;
  DBuf<float> wz32, wy32, wt32;
  // smoother in nested-dissection numbering (fine_order 1): the smoother's
  // matrix F = Q A Q^T (pattern), position -> unknown, and its factors over
  // the dissection tree (or level sweeps in S.L0/S.U0)
  bool fine_nd = false, ftree = false;
  DBuf<int> fperm, frp, fci;
  std::vector<NdNode> fnd_tree;
  TreeSolve tL0, tU0;
  TreeSolve tU0t, tL0t;       // their transposes (adjoint), when both follow the tree
  bool ftree_adj = false;
  DBuf<double> fext, fzp, ftp;
  DBuf<float> fext32, fzp32, ftp32;
  // Krylov workspace
  int mcap = 0;
  size_t ld = 0;
  DBuf<double> V, Z, w, xcol, bcol, coef;
  size_t ldg = 0;
  DBuf<double> gram, gcoef, gdots;  // the basis' Gram matrix (ldg x ldg), corrected coefficients, V^T w_new
  RedWork rw;
  BatchWork bw;                // multi-right-hand-side solve (allocated on first use)
  DBuf<int> abort_flag;
  double* hpin = nullptr;      // pinned host scalars, then two Hessenberg columns (kPinCol each)
  hipEvent_t colev[2] = {nullptr, nullptr};  // a column's copy into hpin finished
  gmg_info info{};
  int log_every = 0;           // GMG_LOG=k prints the residual estimate every k steps
  std::vector<double> hist;    // FGMRES residual estimates of the last solve, per step
  bool force_column_loop = false;  // GMG_COLUMN_LOOP=1: solve several RHS one after another (timing reference)
  int spmv_cap = 4096;         // LDS products per SpMV tile (from A's largest 256-row tile)
  // profiling
  bool prof = false;
  unsigned prof_mask = 0;      // classes that record events (bit c: class c)
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  int64_t pc_launch[PC_COUNT] = {};
  double pc_ms[PC_COUNT] = {}, pc_bytes[PC_COUNT] = {};

  ~Solver() {
    for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (hpin) (void)hipHostFree(hpin);
    for (auto e : colev)
      if (e) (void)hipEventDestroy(e);
  }

  hipEvent_t ev() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    // timing only (read after a stream synchronisation): without the
    // system-scope fence, whose cache write-back cost ~10 us per record
    hipEvent_t e;
    HIPCK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
  }
};

// RAII timing of one launch (or a group) when profiling is on
struct Prof {
  Solver& S;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  Prof(Solver& s_, int c, double b) : S(s_), cls(c), bytes(b) {
    if (S.prof && (S.prof_mask >> cls & 1u)) { a = S.ev(); HIPCK(hipEventRecord(a, S.s)); }
  }
  ~Prof() noexcept(false) {
    if (S.prof && a) {
      hipEvent_t b = S.ev();
      HIPCK(hipEventRecord(b, S.s));
      S.recs.push_back({cls, a, b, bytes});
    }
  }
};

static void prof_flush(Solver& S) {
  if (S.recs.empty()) return;
  HIPCK(hipStreamSynchronize(S.s));
  for (auto& r : S.recs) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, r.a, r.b));
    S.pc_ms[r.cls] += ms;
    S.pc_launch[r.cls] += 1;
    S.pc_bytes[r.cls] += r.bytes;
    S.pool.push_back(r.a);
    S.pool.push_back(r.b);
  }
  S.recs.clear();
}

// ----------------------------------------------------------------- sweeps
// Cut the levels into ranges, each one launch: runs of narrow levels (at
// most wg_chunks chunks, or every level when all_wg) run on one workgroup,
// the others on the whole device.  A run shorter than kMinRun levels joins
// the run before it, so a factor gets a few launches; a one-workgroup run is
// split where its rows would overflow kSweepLdsRows, and a single level that
// alone overflows it runs device-wide.
static void make_segments(Sweep& sw, const std::vector<int>& level_c0, const std::vector<int>& level_e0,
                          int levels, int wg_chunks, bool all_wg) {
  constexpr int kMinRun = 16;
  sw.seg_c0.clear();
  sw.seg_c1.clear();
  sw.seg_e0.clear();
  sw.seg_e1.clear();
  sw.seg_wg.clear();
  std::vector<int> run_l0;
  std::vector<char> run_wg;
  for (int l = 0; l < levels; ++l) {
    const char wg = (all_wg || (level_c0[l + 1] - level_c0[l]) <= wg_chunks) ? 1 : 0;
    if (run_wg.empty() || run_wg.back() != wg) { run_l0.push_back(l); run_wg.push_back(wg); }
  }
  std::vector<int> l0;
  std::vector<char> kind;
  for (size_t r = 0; r < run_l0.size(); ++r) {
    const int len = (r + 1 < run_l0.size() ? run_l0[r + 1] : levels) - run_l0[r];
    if (!l0.empty() && (len < kMinRun || run_wg[r] == kind.back())) continue;
    l0.push_back(run_l0[r]);
    kind.push_back(run_wg[r]);
  }
  auto emit = [&](int la, int lb, char wg) {
    if (level_c0[lb] == level_c0[la]) return;
    sw.seg_c0.push_back(level_c0[la]);
    sw.seg_c1.push_back(level_c0[lb]);
    sw.seg_e0.push_back(level_e0[la]);
    sw.seg_e1.push_back(level_e0[lb]);
    sw.seg_wg.push_back(wg);
  };
  for (size_t g = 0; g < l0.size(); ++g) {
    const int la = l0[g], lb = g + 1 < l0.size() ? l0[g + 1] : levels;
    if (!kind[g]) { emit(la, lb, 0); continue; }
    int start = la;
    for (int l = la; l < lb; ++l) {
      const int rows_l = level_e0[l + 1] - level_e0[l];
      if (rows_l > kSweepLdsRows) {  // too wide for LDS
        emit(start, l, 1);
        emit(l, l + 1, 0);
        start = l + 1;
      } else if (level_e0[l + 1] - level_e0[start] > kSweepLdsRows) {
        emit(start, l, 1);
        start = l;
      }
    }
    emit(start, lb, 1);
  }
}

// Runs f(begin, end, thread) over [0, n) split into one contiguous range per
// host thread (one range when n is small).
template <class F>
static void parallel_ranges(int n, F&& f) {
  const int nt = std::max(1, std::min(host_threads(), n / 4096));
  if (nt == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&f, n, nt, t] { f((int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt), t); });
  for (auto& th : pool) th.join();
}

// Host-to-device copy of a large pageable host array (a factor's entries at
// setup).  The runtime stages a pageable copy through one small pinned buffer,
// a host copy and a DMA at a time (about 11 GB/s measured).  Here up to four
// host threads each copy a contiguous share through two pinned chunks of their
// own, so their host copies run side by side and overlap the DMAs.  The
// chunks are kept for the process and handed out again; the call returns when
// its DMAs have finished (the source may then be freed; the destination is
// ready for work queued on s after the call).
constexpr size_t kStageChunk = (size_t)4 << 20;
constexpr size_t kStageMin = (size_t)8 << 20;  // smaller copies take the runtime's path

static std::mutex g_stage_mu;
static std::vector<void*>* g_stage_free = new std::vector<void*>();  // never freed: pinned for the process

static void* stage_get() {
  {
    std::lock_guard<std::mutex> g(g_stage_mu);
    if (!g_stage_free->empty()) {
      void* p = g_stage_free->back();
      g_stage_free->pop_back();
      return p;
    }
  }
  void* p = nullptr;
  HIPCK(hipHostMalloc(&p, kStageChunk, hipHostMallocPortable));  // any device may use a chunk
  return p;
}
static void stage_put(void* p) {
  std::lock_guard<std::mutex> g(g_stage_mu);
  g_stage_free->push_back(p);
}

template <class T>
static void h2d_large(T* dst, const T* src, size_t n, hipStream_t s) {
  const size_t bytes = n * sizeof(T);
  if (bytes < kStageMin) {
    h2d(dst, src, n, s);
    return;
  }
  const int nt = (int)std::max<size_t>(1, std::min<size_t>({(size_t)4, (size_t)host_threads(), bytes / kStageMin}));
  std::vector<std::exception_ptr> err(nt);
  auto share = [&](int t) {
    const size_t b0 = bytes * t / nt, b1 = bytes * (t + 1) / nt;
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    try {
      int k = 0;
      for (size_t off = b0; off < b1; off += kStageChunk, k ^= 1) {
        const size_t len = std::min(kStageChunk, b1 - off);
        if (!buf[k]) {
          buf[k] = stage_get();
          HIPCK(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        } else {
          HIPCK(hipEventSynchronize(ev[k]));
        }
        std::memcpy(buf[k], reinterpret_cast<const char*>(src) + off, len);
        HIPCK(hipMemcpyAsync(reinterpret_cast<char*>(dst) + off, buf[k], len, hipMemcpyHostToDevice, s));
        HIPCK(hipEventRecord(ev[k], s));
      }
    } catch (...) {
      err[t] = std::current_exception();
    }
    for (int k = 0; k < 2; ++k) {
      if (!ev[k]) continue;
      if (hipEventSynchronize(ev[k]) == hipSuccess) {
        stage_put(buf[k]);  // a chunk whose DMA did not finish is not reused
      } else {
        (void)hipGetLastError();
      }
      (void)hipEventDestroy(ev[k]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(share, t);
  share(0);
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

// Device-to-host copy into a large pageable host array, the reverse of
// h2d_large: each host thread's share comes through two pinned chunks, the
// next chunk's DMA in flight while the current one is copied out.  Returns
// when the data is in dst (work queued on s before the call is waited for).
template <class T>
static void d2h_large(T* dst, const T* src, size_t n, hipStream_t s) {
  const size_t bytes = n * sizeof(T);
  if (bytes < kStageMin) {
    d2h(dst, src, n, s);
    HIPCK(hipStreamSynchronize(s));
    return;
  }
  const int nt = (int)std::max<size_t>(1, std::min<size_t>({(size_t)4, (size_t)host_threads(), bytes / kStageMin}));
  std::vector<std::exception_ptr> err(nt);
  auto share = [&](int t) {
    const size_t b0 = bytes * t / nt, b1 = bytes * (t + 1) / nt;
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    try {
      auto issue = [&](int k, size_t off) {
        if (!buf[k]) {
          buf[k] = stage_get();
          HIPCK(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        }
        const size_t len = std::min(kStageChunk, b1 - off);
        HIPCK(hipMemcpyAsync(buf[k], reinterpret_cast<const char*>(src) + off, len, hipMemcpyDeviceToHost, s));
        HIPCK(hipEventRecord(ev[k], s));
      };
      int k = 0;
      if (b0 < b1) issue(0, b0);
      for (size_t off = b0; off < b1; k ^= 1) {
        const size_t len = std::min(kStageChunk, b1 - off);
        if (off + len < b1) issue(k ^ 1, off + len);
        HIPCK(hipEventSynchronize(ev[k]));
        std::memcpy(reinterpret_cast<char*>(dst) + off, buf[k], len);
        off += len;
      }
    } catch (...) {
      err[t] = std::current_exception();
    }
    for (int k = 0; k < 2; ++k) {
      if (!ev[k]) continue;
      if (hipEventSynchronize(ev[k]) == hipSuccess) {
        stage_put(buf[k]);
      } else {
        (void)hipGetLastError();
      }
      (void)hipEventDestroy(ev[k]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(share, t);
  share(0);
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

// Lay a triangular factor out for the tree solve (k_tree.hip).  Row r's
// entries are q in [rp[r] + skip, rp[r+1]) with column ci[q] and value
// vals[src ? src[q] : q].  Nodes above kTreeMaxRows rows are first cut into
// chains (split_tree).  Returns false (and leaves ts empty) when the factor
// does not follow the tree: an entry outside its row's node must point into a
// descendant node (lower) or an ancestor node (upper).  The host checks the structure and counts the outside
// entries per row; the dense diagonal blocks and the outside-entry lists are
// scattered on the GPU, then the blocks are inverted there.
// The dissection tree with every node cut to at most max_rows rows: a larger
// node (a separator, dense after fill) becomes a chain of consecutive row
// blocks, the first taking the node's children and each next one the block
// before it, the last hanging from the first block of the node's parent.
// Entries between blocks of one node then point into a descendant (lower
// factor) or an ancestor (upper factor), like any other outside entry, so
// the factor still follows the tree.  Node 0 stays the root; heights are
// recomputed.
static std::vector<NdNode> split_tree(const std::vector<NdNode>& t, int max_rows) {
  const int nn = (int)t.size();
  bool any = false;
  for (const NdNode& d : t) any = any || d.hi - d.lo > max_rows;
  if (!any) return t;
  std::vector<int> nb(nn), first(nn);
  int total = 0;
  for (int x = 0; x < nn; ++x) {
    const int sz = t[x].hi - t[x].lo;
    nb[x] = std::max(1, (sz + max_rows - 1) / max_rows);
    first[x] = total;
    total += nb[x];
  }
  // chain of x: ids first[x] + k, k = 0 (bottom) .. nb[x] - 1 (top); the
  // root's top is then moved to id 0
  std::vector<NdNode> out(total);
  for (int x = 0; x < nn; ++x) {
    const int sz = t[x].hi - t[x].lo, b = (sz + nb[x] - 1) / std::max(1, nb[x]);
    for (int k = 0; k < nb[x]; ++k) {
      NdNode& d = out[first[x] + k];
      d.lo = std::min(t[x].hi, t[x].lo + k * b);
      d.hi = std::min(t[x].hi, t[x].lo + (k + 1) * b);
      d.parent = k + 1 < nb[x] ? first[x] + k + 1 : (t[x].parent < 0 ? -1 : first[t[x].parent]);
      d.height = 0;
    }
  }
  const int root = first[0] + nb[0] - 1;
  if (root != 0) {
    std::swap(out[0], out[root]);
    for (NdNode& d : out) {
      if (d.parent == 0) d.parent = root;
      else if (d.parent == root) d.parent = 0;
    }
  }
  // heights: children before parents in a post-order from the root
  std::vector<std::vector<int>> kids(total);
  for (int k = 1; k < total; ++k) kids[out[k].parent].push_back(k);
  std::vector<int> order, st{0};
  while (!st.empty()) {
    const int k = st.back();
    st.pop_back();
    order.push_back(k);
    for (int c : kids[k]) st.push_back(c);
  }
  for (int i = (int)order.size() - 1; i >= 0; --i) {
    const int k = order[i];
    for (int c : kids[k]) out[k].height = std::max(out[k].height, out[c].height + 1);
  }
  return out;
}

static bool build_tree(TreeSolve& ts, const std::vector<NdNode>& tree_in, int n, const std::vector<int>& rp,
                       const std::vector<int>& ci, const std::vector<int>* src, int skip,
                       const std::vector<double>& vals, bool lower, const std::vector<double>* dinv,
                       hipStream_t s) {
  const std::vector<NdNode> tree = split_tree(tree_in, kTreeMaxRows);
  constexpr int kHelperEntries = 256, kHelperRows = 32;
  constexpr int kSliceLgRows = 4;             // rows per slice of a node above 64 rows: 16
  constexpr int kWideRows = 1024, kWideLgRows = 3;  // rows per slice of a node of 1024 rows or more: 8
  constexpr size_t kSmallInvLds = 40 * 1024;  // inversion chunks launched with this much LDS or less first
  const int nn = (int)tree.size();
  if (nn == 0 || n <= 0) return false;
  std::vector<int> node_of(n, -1), nlo(nn), nsz(nn);
  int max_rows = 0, max_h = 0;
  for (int k = 0; k < nn; ++k) {
    const NdNode& d = tree[k];
    if (d.hi - d.lo > kTreeMaxRows) return false;
    nlo[k] = d.lo;
    nsz[k] = d.hi - d.lo;
    max_rows = std::max(max_rows, d.hi - d.lo);
    max_h = std::max(max_h, d.height);
    for (int r = d.lo; r < d.hi; ++r) node_of[r] = k;
  }
  for (int r = 0; r < n; ++r)
    if (node_of[r] < 0) return false;
  // Euler-tour intervals: x is a descendant of y iff tin[y] <= tin[x] < tout[y]
  std::vector<std::vector<int>> kids(nn);
  for (int k = 1; k < nn; ++k) kids[tree[k].parent].push_back(k);
  std::vector<int> tin(nn), tout(nn), st{0}, it(nn, 0);
  int clock = 0;
  tin[0] = clock++;
  while (!st.empty()) {
    const int k = st.back();
    if (it[k] < (int)kids[k].size()) {
      const int c = kids[k][it[k]++];
      tin[c] = clock++;
      st.push_back(c);
    } else {
      tout[k] = clock;
      st.pop_back();
    }
  }
  auto desc = [&](int x, int y) { return tin[y] <= tin[x] && tin[x] < tout[y]; };
  // outside entries per row, and the structure check
  std::vector<int> erp(n + 1, 0);
  std::vector<char> bad(std::max(1, std::min(host_threads(), n / 4096)), 0);
  parallel_ranges(n, [&](int r0, int r1, int t) {
    for (int r = r0; r < r1; ++r) {
      const int a = node_of[r];
      int cnt = 0;
      for (int q = rp[r] + skip; q < rp[r + 1]; ++q) {
        const int b = node_of[ci[q]];
        if (b == a) continue;
        if (!(lower ? desc(b, a) : desc(a, b))) bad[t] = 1;
        ++cnt;
      }
      erp[r + 1] = cnt;
    }
  });
  for (char b : bad)
    if (b) return false;
  for (int r = 0; r < n; ++r) erp[r + 1] += erp[r];
  std::vector<int64_t> boff(nn, 0), node_ext(nn, 0);
  int64_t total = 0;
  for (int k = 0; k < nn; ++k) {
    boff[k] = total;
    total += (int64_t)nsz[k] * nsz[k];
    node_ext[k] = erp[tree[k].hi] - erp[tree[k].lo];
  }
  // tasks: nodes by height (lower: ascending, upper: descending), each node's
  // helpers (slices of about kHelperEntries outside entries) before it
  std::vector<int> order;
  for (int k = 0; k < nn; ++k)
    if (tree[k].hi > tree[k].lo) order.push_back(k);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return lower ? tree[x].height < tree[y].height : tree[x].height > tree[y].height;
  });
  std::vector<int> task;
  int pair_open = -1;  // offset of a pair task whose second half is free
  for (int k : order) {
    const NdNode& d = tree[k];
    const bool has_ext = node_ext[k] > 0;
    if (has_ext) {
      int r = d.lo;
      while (r < d.hi) {
        int r1 = r, ents = 0, longest = 0;
        while (r1 < d.hi && r1 - r < kHelperRows && (ents < kHelperEntries || r1 == r)) {
          const int e = erp[r1 + 1] - erp[r1];
          ents += e;
          longest = std::max(longest, e);
          ++r1;
        }
        int lg = 0;
        while ((1 << lg) * 8 < longest && lg < 6) ++lg;
        task.insert(task.end(), {0, d.lo, d.hi - d.lo, r, r1, k, 1, lg});
        r = r1;
      }
    }
    // the node's slices: one for a leaf-sized block, else kSliceRows rows each
    const int sz = d.hi - d.lo;
    const int lgR = sz <= 64 ? 6 : sz >= kWideRows ? kWideLgRows : kSliceLgRows, R = 1 << lgR;
    const int nsl = (sz + R - 1) / R;
    if (lower && !has_ext && sz <= 64) {
      // no outside entries: the node waits on nothing, so it may share the
      // workgroup of an earlier one like it (a pair task, one node per half)
      if (pair_open >= 0) {
        task[pair_open + 4] = d.lo;
        task[pair_open + 5] = sz;
        task[pair_open + 6] = k;
        pair_open = -1;
      } else {
        pair_open = (int)task.size();
        task.insert(task.end(), {2, d.lo, sz, k, 0, 0, k, 0});
      }
      continue;
    }
    for (int q = 0; q < nsl; ++q)
      task.insert(task.end(), {1, d.lo, sz, q * R, std::min(sz, (q + 1) * R), k, (has_ext ? 1 : 0) | lgR << 1, nsl});
  }
  // inversion tasks: W-column chunks of every node, small-LDS ones first
  std::vector<int> itask[2];
  size_t ilds[2] = {0, 0};
  for (int k = 0; k < nn; ++k) {
    const int sz = tree[k].hi - tree[k].lo;
    if (sz == 0) continue;
    const int lgW = tree_inv_width(sz);
    const size_t need = tree_inv_lds(sz, lgW);
    const int cls = need <= kSmallInvLds ? 0 : 1;
    ilds[cls] = std::max(ilds[cls], need);
    for (int c0 = 0; c0 < sz; c0 += 1 << lgW) itask[cls].insert(itask[cls].end(), {tree[k].lo, sz, c0, k, lgW, 0, 0, 0});
  }
  ts.lower = lower;
  ts.has_diag = dinv != nullptr;
  ts.ntasks = (int)task.size() / 8;
  ts.max_rows = max_rows;
  ts.heights = max_h + 1;
  const size_t ne = (size_t)erp[n];
  const size_t nent = (size_t)rp[n];
  ts.task.alloc(task.size());
  ts.erp.alloc(n + 1);
  ts.ecol.alloc(ne > 0 ? ne : 1);
  ts.eval.alloc(ne > 0 ? ne : 1);
  ts.eval32.alloc(ne > 0 ? ne : 1);
  ts.boff.alloc(nn);
  ts.ncount.alloc(nn);
  ts.inv.alloc(total > 0 ? total : 1);
  ts.inv32.alloc(total > 0 ? total : 1);
  h2d(ts.task.p, task.data(), task.size(), s);
  h2d(ts.erp.p, erp.data(), n + 1, s);
  h2d(ts.boff.p, boff.data(), nn, s);
  HIPCK(hipMemsetAsync(ts.ncount.p, 0, sizeof(int) * nn, s));
  {
    // the factor's rows on the device, values in entry order
    DBuf<int> drp, dci, dnode, dlo, dsz;
    DBuf<double> dv, dblk, ddinv;
    DBuf<int> dit[2];
    drp.alloc(n + 1);
    dci.alloc(nent > 0 ? nent : 1);
    dv.alloc(nent > 0 ? nent : 1);
    dnode.alloc(n);
    dlo.alloc(nn);
    dsz.alloc(nn);
    h2d(drp.p, rp.data(), n + 1, s);
    h2d_large(dci.p, ci.data(), nent, s);
    std::vector<double> vq;
    if (src) {
      vq.resize(nent);
      parallel_ranges((int)nent, [&](int q0, int q1, int) {
        for (int q = q0; q < q1; ++q) vq[q] = vals[(*src)[q]];
      });
      h2d_large(dv.p, vq.data(), nent, s);
    } else {
      h2d_large(dv.p, vals.data(), nent, s);
    }
    h2d(dnode.p, node_of.data(), n, s);
    h2d(dlo.p, nlo.data(), nn, s);
    h2d(dsz.p, nsz.data(), nn, s);
    dblk.alloc(total > 0 ? total : 1);
    HIPCK(hipMemsetAsync(dblk.p, 0, sizeof(double) * (total > 0 ? total : 1), s));
    launch_tree_fill(n, drp.p, dci.p, dv.p, skip, dnode.p, dlo.p, dsz.p, ts.boff.p, ts.erp.p, dblk.p, ts.ecol.p,
                     ts.eval.p, s);
    if (dinv) {
      ddinv.alloc(n);
      h2d(ddinv.p, dinv->data(), n, s);
    }
    HIPCK(hipMemsetAsync(ts.inv.p, 0, sizeof(double) * (total > 0 ? total : 1), s));
    for (int c = 0; c < 2; ++c) {
      if (itask[c].empty()) continue;
      dit[c].alloc(itask[c].size());
      h2d(dit[c].p, itask[c].data(), itask[c].size(), s);
      launch_tree_invert(ts, dit[c].p, (int)itask[c].size() / 8, ilds[c], dblk.p, dinv ? ddinv.p : nullptr,
                         ts.inv.p, s);
    }
    launch_cast_f32(ts.eval.p, ts.eval32.p, ne, s);
    launch_cast_f32(ts.inv.p, ts.inv32.p, total, s);
    HIPCK(hipStreamSynchronize(s));  // host vectors and staging buffers go out of scope
  }
  return true;
}

// Build a sweep from host dependency lists.  dep_rp/dep_ci/dep_src list, per
// row, the dependency columns and the index of each value in `src_vals`
// (device) or the value itself (host_vals, when src_vals is null).
static void build_sweep(Sweep& sw, int n, const std::vector<int>& dep_rp, const std::vector<int>& dep_ci,
                        const std::vector<int>& dep_src, const std::vector<double>* host_vals,
                        const double* src_vals_dev, bool lower, bool has_diag,
                        const std::vector<double>* host_dinv, const double* dev_dinv, int wg_chunks,
                        bool all_wg, hipStream_t s) {
  std::vector<int> sched, lptr;
  int levels = 0;
  make_schedule(dep_rp, dep_ci, lower, sched, lptr, &levels);
  std::vector<int> rows, chunk, level_c0(levels + 1, 0), level_e0(levels + 1, 0);
  rows.reserve(n);
  for (int l = 0; l < levels; ++l) {
    level_c0[l] = (int)chunk.size() / 3;
    level_e0[l] = (int)rows.size();
    const int first = (int)rows.size();
    int maxdeps = 0;
    for (int p = lptr[l]; p < lptr[l + 1]; ++p) {
      const int r = sched[p];
      if (r < 0) continue;
      rows.push_back(r);
      maxdeps = std::max(maxdeps, dep_rp[r + 1] - dep_rp[r]);
    }
    // lanes per row: enough that one lane reads at most one batch of 8 entries
    int lg = 0;
    while ((1 << lg) * 8 < maxdeps && lg < 6) ++lg;
    const int per = 64 >> lg;
    const int cnt = (int)rows.size() - first;
    for (int c = 0; c < cnt; c += per) {
      chunk.push_back(first + c);
      chunk.push_back(std::min(per, cnt - c));
      chunk.push_back(lg);
    }
  }
  level_c0[levels] = (int)chunk.size() / 3;
  level_e0[levels] = (int)rows.size();
  make_segments(sw, level_c0, level_e0, levels, wg_chunks, all_wg);
  sw.lvl_c0 = level_c0;
  const int ne_rows = (int)rows.size();
  std::vector<int> dp(ne_rows + 1, 0);
  for (int e = 0; e < ne_rows; ++e) dp[e + 1] = dp[e] + dep_rp[rows[e] + 1] - dep_rp[rows[e]];
  const int64_t ne = dp[ne_rows];
  std::vector<int> dcol(ne > 0 ? ne : 1), dsrc(ne > 0 ? ne : 1);
  std::vector<double> dval_h;
  if (host_vals) dval_h.resize(ne > 0 ? ne : 1);
  for (int e = 0; e < ne_rows; ++e) {
    int o = dp[e];
    for (int q = dep_rp[rows[e]]; q < dep_rp[rows[e] + 1]; ++q, ++o) {
      dcol[o] = dep_ci[q];
      dsrc[o] = dep_src[q];
      if (host_vals) dval_h[o] = (*host_vals)[dep_src[q]];
    }
  }
  sw.n = n;
  sw.nchunks = (int)chunk.size() / 3;
  sw.levels = levels;
  sw.nnz = ne;
  sw.has_diag = has_diag;
  sw.chunk.alloc(chunk.size() > 0 ? chunk.size() : 1);
  sw.rows.alloc(ne_rows > 0 ? ne_rows : 1);
  sw.dp.alloc(ne_rows + 1);
  sw.dcol.alloc(ne > 0 ? ne : 1);
  sw.dval.alloc(ne > 0 ? ne : 1);
  h2d(sw.chunk.p, chunk.data(), chunk.size(), s);
  h2d(sw.rows.p, rows.data(), ne_rows, s);
  h2d(sw.dp.p, dp.data(), ne_rows + 1, s);
  h2d(sw.dcol.p, dcol.data(), ne, s);
  {
    // LDS slots of the dependencies of one-workgroup ranges
    bool any = false;
    for (char w : sw.seg_wg) any = any || w;
    if (any) {
      std::vector<int> pos(n > 0 ? n : 1, -1), dslot(ne > 0 ? ne : 1, 0);
      for (int e = 0; e < ne_rows; ++e) pos[rows[e]] = e;
      for (size_t g = 0; g < sw.seg_wg.size(); ++g) {
        if (!sw.seg_wg[g]) continue;
        const int e0 = sw.seg_e0[g], e1 = sw.seg_e1[g];
        for (int e = e0; e < e1; ++e)
          for (int q = dp[e]; q < dp[e + 1]; ++q) {
            const int c = dcol[q], pc = pos[c];
            dslot[q] = (pc >= e0 && pc < e1) ? pc - e0 : -1 - c;
          }
      }
      sw.dslot.alloc(ne > 0 ? ne : 1);
      h2d(sw.dslot.p, dslot.data(), ne, s);
    }
  }
  if (host_vals) {
    h2d(sw.dval.p, dval_h.data(), ne, s);
  } else {
    DBuf<int> src;
    src.alloc(ne > 0 ? ne : 1);
    h2d(src.p, dsrc.data(), ne, s);
    launch_gather_f64(src_vals_dev, src.p, sw.dval.p, ne, s);
    HIPCK(hipStreamSynchronize(s));
  }
  sw.dval32.alloc(ne > 0 ? ne : 1);
  launch_cast_f32(sw.dval.p, sw.dval32.p, ne, s);
  if (has_diag) {
    sw.dinv.alloc(n > 0 ? n : 1);
    sw.dinv32.alloc(n > 0 ? n : 1);
    if (host_dinv) h2d(sw.dinv.p, host_dinv->data(), n, s);
    else d2d(sw.dinv.p, dev_dinv, n, s);
    launch_cast_f32(sw.dinv.p, sw.dinv32.p, n, s);
  }
  sw.ticket.alloc(1);
  launch_fill_u32(sw.ticket.p, 0u, 1, s);
  sw.ticket_base = 0;
  {
    // a few levels of look-ahead: more resident waves would only poll
    const double per_level = levels > 0 ? (double)sw.nchunks / levels : 1.0;
    sw.waves = std::min(2048, std::max(16, (int)std::ceil(4.0 * per_level)));
  }
  // single-CU form when every level has at most 1024 rows, every row at most
  // 4 entries, and every entry points at one of the two previous levels
  sw.cu.reset();
  {
    std::vector<int> lev(n > 0 ? n : 1, 0), pos(n > 0 ? n : 1, 0), ulptr(levels + 1, 0);
    bool ok = levels > 0 && levels <= 16000;  // level bounds are staged in LDS
    int width = 1;
    for (int l = 0; l < levels && ok; ++l) {
      int cnt = 0;
      for (int p = lptr[l]; p < lptr[l + 1]; ++p) {
        const int r = sched[p];
        if (r < 0) continue;
        lev[r] = l;
        pos[r] = cnt++;
        width = std::max(width, dep_rp[r + 1] - dep_rp[r]);
      }
      ulptr[l + 1] = ulptr[l] + cnt;
      if (cnt > 1024) ok = false;
    }
    if (width > 4) ok = false;
    for (int e = 0; e < ne_rows && ok; ++e) {
      const int r = rows[e];
      for (int q = dep_rp[r]; q < dep_rp[r + 1]; ++q)
        if (lev[dep_ci[q]] < lev[r] - 2) { ok = false; break; }
    }
    if (ok) {
      const int W = width <= 2 ? width : 4;  // kernel instances: 1, 2, 3->4, 4
      const int Wk = width == 3 ? 3 : W;
      std::unique_ptr<CuSweep> cs(new CuSweep());
      cs->n = ne_rows;
      cs->levels = levels;
      cs->width = Wk;
      cs->has_diag = has_diag;
      // one extra (dummy) entry at index n: zero operands, read by idle threads
      std::vector<int> wslot((size_t)(ne_rows + 1) * Wk, 3 * 1024), wsrc((size_t)(ne_rows + 1) * Wk, -1);
      for (int e = 0; e < ne_rows; ++e) {
        const int r = rows[e];
        int k = 0;
        for (int q = dep_rp[r]; q < dep_rp[r + 1]; ++q, ++k) {
          const int c = dep_ci[q];
          wslot[(size_t)e * Wk + k] = (lev[c] % 3) * 1024 + pos[c];
          wsrc[(size_t)e * Wk + k] = dp[e] + k;  // index into sw.dval (entry order)
        }
      }
      cs->lptr.alloc(levels + 1);
      cs->rows.alloc(ne_rows > 0 ? ne_rows : 1);
      cs->wslot.alloc(wslot.size() > 0 ? wslot.size() : 1);
      h2d(cs->lptr.p, ulptr.data(), levels + 1, s);
      h2d(cs->rows.p, rows.data(), ne_rows, s);
      h2d(cs->wslot.p, wslot.data(), wslot.size(), s);
      // values: gather from the entry-ordered dval; padding entries get 0
      std::vector<double> zero(1, 0.0);
      DBuf<double> withzero;
      withzero.alloc(ne + 1);
      d2d(withzero.p, sw.dval.p, ne, s);
      h2d(withzero.p + ne, zero.data(), 1, s);
      for (auto& x : wsrc)
        if (x < 0) x = (int)ne;
      DBuf<int> dsrc2;
      dsrc2.alloc(wsrc.size() > 0 ? wsrc.size() : 1);
      h2d(dsrc2.p, wsrc.data(), wsrc.size(), s);
      cs->wval.alloc(wsrc.size() > 0 ? wsrc.size() : 1);
      cs->wval32.alloc(wsrc.size() > 0 ? wsrc.size() : 1);
      launch_gather_f64(withzero.p, dsrc2.p, cs->wval.p, (int64_t)wsrc.size(), s);
      launch_cast_f32(cs->wval.p, cs->wval32.p, wsrc.size(), s);
      if (has_diag) {
        cs->dinv_e.alloc(ne_rows + 1);
        cs->dinv_e32.alloc(ne_rows + 1);
        launch_fill_f64_bits(cs->dinv_e.p + ne_rows, 0ULL, 1, s);
        launch_gather_f64(sw.dinv.p, cs->rows.p, cs->dinv_e.p, ne_rows, s);
        launch_cast_f32(cs->dinv_e.p, cs->dinv_e32.p, ne_rows + 1, s);
      }
      HIPCK(hipStreamSynchronize(s));
      sw.cu = std::move(cs);
    }
  }
  HIPCK(hipStreamSynchronize(s));  // host vectors above go out of scope
}

__global__ void k_recip_diag(int n, const double* __restrict__ a, const int* __restrict__ dpos,
                             double* __restrict__ dinv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dinv[i] = 1.0 / a[dpos[i]];
}

static double sweep_bytes(const Sweep& sw, size_t sz, size_t szr, bool reset) {
  // structure + dependency values + rhs + result write + result reads + diag
  return (double)sw.nnz * (4 + sz) + (double)sw.n * (8 + szr + 2 * sz + (sw.has_diag ? sz : 0) + (reset ? szr : 0));
}

static void check_abort(Solver& S) {
  int f = 0;
  d2h(&f, S.abort_flag.p, 1, S.s);
  HIPCK(hipStreamSynchronize(S.s));
  if (f) {
    launch_fill_u32(reinterpret_cast<unsigned*>(S.abort_flag.p), 0u, 1, S.s);
    fail(GMG_ERR_STALLED, "a triangular-sweep dependency wait timed out");
  }
}

// One triangular sweep of a factor: the single-CU kernel when the factor has
// one and it is enabled, else the synchronisation-free kernel over the
// factor's level segments (one workgroup or the whole device each).
template <class T>
static void run_tri(Solver& S, Sweep& sw, const void* rhs, bool rhs_f64, T* out, T* reset) {
  constexpr bool F32 = sizeof(T) == 4;
  if (sw.cu && (S.opt.sweep_kernel == 0 || S.opt.sweep_kernel == 3)) {
    CuSweep& c = *sw.cu;
    launch_cu_sweep<T>(c, F32 ? (const T*)c.wval32.p : (const T*)c.wval.p,
                       F32 ? (const T*)c.dinv_e32.p : (const T*)c.dinv_e.p, rhs, rhs_f64, out, reset,
                       F32 ? (T*)S.cu_rhs32.p : (T*)S.cu_rhs.p, F32 ? (T*)S.cu_out32.p : (T*)S.cu_out.p, S.s);
    return;
  }
  const T* di = sw.has_diag ? (F32 ? (const T*)sw.dinv32.p : (const T*)sw.dinv.p) : nullptr;
  if (S.opt.sweep_kernel == 0 && sw.levels <= kLevelLaunchMax && (int)sw.lvl_c0.size() == sw.levels + 1) {
    // a few wide levels (colour classes): one plain launch per level
    launch_sweep_levels<T>(sw, F32 ? (const T*)sw.dval32.p : (const T*)sw.dval.p, di, rhs, rhs_f64, out, reset, S.s);
    return;
  }
  const int waves = S.opt.sweep_waves > 0 ? S.opt.sweep_waves : sw.waves;
  launch_sweep<T>(sw, F32 ? (const T*)sw.dval32.p : (const T*)sw.dval.p, di, rhs, rhs_f64, out, reset, waves,
                  S.opt.sweep_kernel == 1, S.abort_flag.p, S.s);
}

static void reset_cycle_buffers(Solver& S) {
  hipStream_t s = S.s;
  if (S.wave) {
    launch_fill_f64_bits(S.wy.p, kSent64, S.wg.total, s);
    launch_fill_f64_bits(S.wt.p, kSent64, S.wg.total, s);
    launch_fill_f32_bits(S.wy32.p, kSent32, S.wg.total, s);
    launch_fill_f32_bits(S.wt32.p, kSent32, S.wg.total, s);
  }
  if (S.tree) {
    launch_fill_f64_bits(S.text.p, kSent64, S.nc, s);
    launch_fill_f32_bits(S.text32.p, kSent32, S.nc, s);
    for (TreeSolve* t : {&S.tLc, &S.tUc, &S.tUct, &S.tLct})
      if (t->ncount.p) launch_fill_f32_bits(reinterpret_cast<float*>(t->ncount.p), 0u, t->ncount.n, s);
  }
  if (S.ftree) {
    launch_fill_f64_bits(S.fext.p, kSent64, S.n, s);
    launch_fill_f32_bits(S.fext32.p, kSent32, S.n, s);
    for (TreeSolve* t : {&S.tL0, &S.tU0})
      if (t->ncount.p) launch_fill_f32_bits(reinterpret_cast<float*>(t->ncount.p), 0u, t->ncount.n, s);
  }
  if (S.fine_nd) {
    launch_fill_f64_bits(S.ftp.p, kSent64, S.n, s);
    launch_fill_f32_bits(S.ftp32.p, kSent32, S.n, s);
  }
  launch_fill_f64_bits(S.y.p, kSent64, S.n, s);
  launch_fill_f64_bits(S.t.p, kSent64, S.n, s);
  launch_fill_f64_bits(S.yc.p, kSent64, S.nc, s);
  launch_fill_f64_bits(S.ec.p, kSent64, S.nc, s);
  launch_fill_f32_bits(S.y32.p, kSent32, S.n, s);
  launch_fill_f32_bits(S.t32.p, kSent32, S.n, s);
  launch_fill_f32_bits(S.yc32.p, kSent32, S.nc, s);
  launch_fill_f32_bits(S.ec32.p, kSent32, S.nc, s);
  launch_fill_f64_bits(S.auc.p, kSent64, S.nc, s);
  launch_fill_f64_bits(S.aec.p, kSent64, S.nc, s);
  launch_fill_f64_bits(S.aw.p, kSent64, S.n, s);
  launch_fill_f64_bits(S.at.p, kSent64, S.n, s);
}

// ------------------------------------------------------ preconditioner apply
// t = S^{-1} z, the ILU(0) smoothing step (precision T; t is the output of a
// triangular sweep, so it holds the sentinel on entry)
template <class T>
static void smooth_apply(Solver& S, const double* z, T* t) {
  constexpr bool F32 = sizeof(T) == 4;
  hipStream_t s = S.s;
  T* y = F32 ? (T*)S.y32.p : (T*)S.y.p;
  const size_t sz = sizeof(T);
  if (S.wave) {
    Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.L0, sz, 8, false) + sweep_bytes(S.U0, sz, sz, true));
    launch_wave_pair<T>(S.wg, S.wL0, S.wU0, z, true, F32 ? (T*)S.wz32.p : (T*)S.wz.p, F32 ? (T*)S.wy32.p : (T*)S.wy.p,
                        F32 ? (T*)S.wt32.p : (T*)S.wt.p, t, S.abort_flag.p, s);
  } else if (S.fine_nd) {
    // t = Q^T U0^{-1} L0^{-1} Q z
    Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.L0, sz, sz, false) + sweep_bytes(S.U0, sz, sz, true) +
                                 (double)S.n * (2 * 4 + 8 + 3 * sz));
    T* zp = F32 ? (T*)S.fzp32.p : (T*)S.fzp.p;
    T* tp = F32 ? (T*)S.ftp32.p : (T*)S.ftp.p;
    launch_perm_gather<T>(S.n, S.fperm.p, z, zp, s);
    if (S.ftree) {
      T* ext = F32 ? (T*)S.fext32.p : (T*)S.fext.p;
      launch_tree<T>(S.tL0, zp, false, y, nullptr, ext, S.abort_flag.p, s);
      launch_tree<T>(S.tU0, y, false, tp, y, ext, S.abort_flag.p, s);
    } else {
      run_tri<T>(S, S.L0, zp, false, y, nullptr);
      run_tri<T>(S, S.U0, y, false, tp, y);
    }
    launch_perm_scatter<T>(S.n, S.fperm.p, tp, t, s);
  } else {
    {
      Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.L0, sz, 8, false));
      run_tri<T>(S, S.L0, z, true, y, nullptr);
    }
    {
      Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.U0, sz, sz, true));
      run_tri<T>(S, S.U0, y, false, t, y);
    }
  }
}

// ec = A~_c^{-1} rc, the inexact coarse solve (precision T; ec holds the
// sentinel on entry, as the restriction leaves it)
template <class T>
static void coarse_apply(Solver& S, T* rc, T* ec) {
  constexpr bool F32 = sizeof(T) == 4;
  hipStream_t s = S.s;
  T* yc = F32 ? (T*)S.yc32.p : (T*)S.yc.p;
  const size_t sz = sizeof(T);
  if (S.opt.coarse_mode == 0 && S.tree) {
    T* ext = F32 ? (T*)S.text32.p : (T*)S.text.p;
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Lc, sz, sz, false));
      launch_tree<T>(S.tLc, rc, false, yc, nullptr, ext, S.abort_flag.p, s);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Uc, sz, sz, true));
      launch_tree<T>(S.tUc, yc, false, ec, yc, ext, S.abort_flag.p, s);
    }
  } else if (S.opt.coarse_mode == 0) {
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Lc, sz, sz, false));
      run_tri<T>(S, S.Lc, rc, false, yc, nullptr);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Uc, sz, sz, true));
      run_tri<T>(S, S.Uc, yc, false, ec, yc);
    }
  } else if (S.opt.coarse_mode == 3) {
    // e_c = A_c^{-1} r_c with the dense inverse
    Prof p(S, PC_SWEEP_COARSE, (double)S.nc * S.nc * sz + (double)S.nc * 2 * sz);
    launch_dense_gemv<T>(S.nc, S.cnp, F32 ? (const T*)S.cinv32.p : (const T*)S.cinv.p, rc, ec, s);
  } else if (S.opt.coarse_mode == 2) {
    // e_c = M r_c with the sparse approximate inverse
    Prof p(S, PC_SWEEP_COARSE, (double)S.dMc.nnz * (4 + sz) + (double)S.nc * (4 + 2 * sz));
    launch_spmv<T>(S.nc, S.dMc.rp.p, S.dMc.ci.p, F32 ? (const T*)S.dMc.v32.p : (const T*)S.dMc.v.p, rc, ec, s);
  } else {
    if (F32) fail(GMG_ERR_INVALID_ARG, "coarse_mode 1 runs in FP64 only");
    // Jacobi sweeps on each factor: y <- rc - (L~ - I) y from y = rc, then
    // e <- D^{-1} (y - (U~ - D) e) from e = D^{-1} y
    Prof p(S, PC_SWEEP_COARSE, 0.0);
    const double* rcd = (const double*)rc;
    double* a0 = (double*)yc;
    double* a1 = S.jtmp.p;
    d2d(a0, rcd, S.nc, s);
    for (int k = 0; k < S.opt.coarse_sweeps; ++k) {
      launch_jacobi(S.nc, S.dLc.rp.p, S.dLc.ci.p, S.dLc.v.p, nullptr, rcd, a0, a1, s);
      std::swap(a0, a1);
    }
    double* e0 = (double*)ec;
    double* e1 = a1;  // the L iterate buffer not holding the result
    launch_jacobi(S.nc, S.dUc.rp.p, S.dUc.ci.p, S.dUc.v.p, S.ucdinv.p, a0, S.jzero.p, e0, s);
    for (int k = 0; k < S.opt.coarse_sweeps; ++k) {
      launch_jacobi(S.nc, S.dUc.rp.p, S.dUc.ci.p, S.dUc.v.p, S.ucdinv.p, a0, e0, e1, s);
      std::swap(e0, e1);
    }
    if (e0 != (double*)ec) d2d((double*)ec, e0, S.nc, s);
  }
}

// q = B~^{-1} z: t = U0^{-1} L0^{-1} z; r = z - A t; rc = P^T r;
// ec = U~^{-1} L~^{-1} rc; q = t + P ec  (precision T)
template <class T>
static void vcycle(Solver& S, const double* z, double* q) {
  constexpr bool F32 = sizeof(T) == 4;
  hipStream_t s = S.s;
  T* t = F32 ? (T*)S.t32.p : (T*)S.t.p;
  T* r = F32 ? (T*)S.r32.p : (T*)S.r.p;
  T* rc = F32 ? (T*)S.rc32.p : (T*)S.rc.p;
  T* ec = F32 ? (T*)S.ec32.p : (T*)S.ec.p;
  const T* Av = F32 ? (const T*)S.A.v32.p : (const T*)S.A.v.p;
  const size_t sz = sizeof(T);
  smooth_apply<T>(S, z, t);
  {
    Prof p(S, PC_RESID_RESTRICT, (double)S.nnz * (4 + sz) + (double)S.n * (4 + 8 + 3 * sz + 4) +
                                     (double)S.nc * (4 + 2 * sz));
    launch_resid_fine<T>(S.n, S.A.rp.p, S.A.ci.p, Av, t, z, r, s, S.spmv_cap);
    launch_restrict<T>(S.nc, S.aptr.p, S.amem.p, r, rc, ec, 0, s);
  }
  coarse_apply<T>(S, rc, ec);
  {
    // t is polled for (and so reset to the sentinel) only when the level
    // sweeps produce it; the wavefront and permuted smoothers write it plainly
    const bool reset_t = !S.wave && !S.fine_nd;
    Prof p(S, PC_PROLONG, (double)S.n * (4 + (reset_t ? 2 : 1) * sz + 8) + (double)S.nc * sz);
    launch_prolong<T>(S.n, S.agg.p, t, ec, q, 0, s, reset_t);
  }
}

static std::vector<int> to_host_int(const int* d, size_t n, hipStream_t s);
static void build_wave(WaveSweep& f, const WaveGrid& g, const std::vector<int>& dep_rp,
                       const std::vector<int>& dep_ci, const std::vector<int>& dep_src, bool lower,
                       const double* vals_dev, int64_t nvals, const double* dinv_dev, int n, hipStream_t s);

// The transposed fine and coarse factors of the adjoint cycle, built on the
// first adjoint use (a forward-only caller never pays for them).
static void ensure_adjoint(Solver& S) {
  if (S.adj_ready) return;
  hipStream_t s = S.s;
  const int n = S.n, nc = S.nc;
  const int64_t nnz64 = S.nnz;
  const gmg_options& o = S.opt;
  {
    // row j of U0^T lists i < j with (i, j) in strict U; of L0^T lists i > j
    // with (i, j) in strict L; src: the entry of the factored matrix (A, or
    // F = Q A Q^T for the reordered smoothers) that holds the value
    std::vector<int> hat_rp, hat_ci, hat_src;
    if (!S.fine_nd) {
      hat_rp = to_host_int(S.AT.rp.p, n + 1, s);
      hat_ci = to_host_int(S.AT.ci.p, nnz64, s);
      hat_src = to_host_int(S.at_src.p, nnz64, s);
    } else {
      DBuf<int> ftrp, ftci, ftsrc;
      transpose_csr(n, n, nnz64, S.frp.p, S.fci.p, nullptr, ftrp, ftci, nullptr, &ftsrc, s);
      hat_rp = to_host_int(ftrp.p, n + 1, s);
      hat_ci = to_host_int(ftci.p, nnz64, s);
      hat_src = to_host_int(ftsrc.p, nnz64, s);
      HIPCK(hipStreamSynchronize(s));
    }
    HIPCK(hipStreamSynchronize(s));
    std::vector<int> ut_rp(n + 1, 0), ut_ci, ut_src, lt_rp(n + 1, 0), lt_ci, lt_src;
    for (int j = 0; j < n; ++j) {
      for (int q = hat_rp[j]; q < hat_rp[j + 1]; ++q) {
        const int i = hat_ci[q], p = hat_src[q];
        if (i < j) { ut_ci.push_back(i); ut_src.push_back(p); }
        else if (i > j) { lt_ci.push_back(i); lt_src.push_back(p); }
      }
      ut_rp[j + 1] = (int)ut_ci.size();
      lt_rp[j + 1] = (int)lt_ci.size();
    }
    S.U0t.n = S.L0t.n = n;
    S.U0t.nnz = (int64_t)ut_ci.size();
    S.L0t.nnz = (int64_t)lt_ci.size();
    S.U0t.has_diag = true;
    S.ftree_adj = false;
    if (S.wave) {
      build_wave(S.wU0t, S.wg, ut_rp, ut_ci, ut_src, true, S.ilu.p, nnz64, S.u0dinv.p, n, s);
      build_wave(S.wL0t, S.wg, lt_rp, lt_ci, lt_src, false, S.ilu.p, nnz64, nullptr, n, s);
    } else {
      if (S.ftree) {
        // the transposes of factors that follow the dissection tree follow it
        // too (checked all the same)
        std::vector<double> hilu(nnz64), hud(n);
        d2h(hilu.data(), S.ilu.p, nnz64, s);
        d2h(hud.data(), S.u0dinv.p, n, s);
        HIPCK(hipStreamSynchronize(s));
        S.ftree_adj = build_tree(S.tU0t, S.fnd_tree, n, ut_rp, ut_ci, &ut_src, 0, hilu, true, &hud, s) &&
                      build_tree(S.tL0t, S.fnd_tree, n, lt_rp, lt_ci, &lt_src, 0, hilu, false, nullptr, s);
        if (!S.ftree_adj) {
          S.tU0t = TreeSolve();
          S.tL0t = TreeSolve();
        }
      }
      if (!S.ftree_adj) {
        build_sweep(S.U0t, n, ut_rp, ut_ci, ut_src, nullptr, S.ilu.p, true, true, nullptr, S.u0dinv.p, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
        build_sweep(S.L0t, n, lt_rp, lt_ci, lt_src, nullptr, S.ilu.p, false, false, nullptr, nullptr, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
      } else {
        S.U0t.levels = S.L0t.levels = S.tU0t.heights;
      }
    }
  }
  if (o.coarse_mode == 0) {
    // U~^T row j lists i < j (strict part), L~^T row j lists i > j
    const HCsr &L = S.hLc, &U = S.hUc;
    std::vector<double> udinv(nc);
    std::vector<int> uct_cnt(nc + 1, 0), lct_cnt(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
      udinv[i] = 1.0 / U.v[U.rp[i]];
      for (int q = U.rp[i] + 1; q < U.rp[i + 1]; ++q) uct_cnt[U.ci[q] + 1]++;
      for (int q = L.rp[i]; q < L.rp[i + 1]; ++q) lct_cnt[L.ci[q] + 1]++;
    }
    for (int j = 0; j < nc; ++j) { uct_cnt[j + 1] += uct_cnt[j]; lct_cnt[j + 1] += lct_cnt[j]; }
    std::vector<int> uct_ci(uct_cnt[nc]), uct_src(uct_cnt[nc]), lct_ci(lct_cnt[nc]), lct_src(lct_cnt[nc]);
    std::vector<int> fu(uct_cnt.begin(), uct_cnt.end() - 1), fl(lct_cnt.begin(), lct_cnt.end() - 1);
    for (int i = 0; i < nc; ++i) {
      for (int q = U.rp[i] + 1; q < U.rp[i + 1]; ++q) {
        const int o2 = fu[U.ci[q]]++;
        uct_ci[o2] = i;
        uct_src[o2] = q;
      }
      for (int q = L.rp[i]; q < L.rp[i + 1]; ++q) {
        const int o2 = fl[L.ci[q]]++;
        lct_ci[o2] = i;
        lct_src[o2] = q;
      }
    }
    // the transposes of tree-following factors follow the tree too (an entry
    // into a descendant becomes one into an ancestor); checked all the same
    S.tree_adj = S.tree && build_tree(S.tUct, S.nd_tree, nc, uct_cnt, uct_ci, &uct_src, 0, U.v, true, &udinv, s) &&
                 build_tree(S.tLct, S.nd_tree, nc, lct_cnt, lct_ci, &lct_src, 0, L.v, false, nullptr, s);
    if (S.tree_adj) {
      S.Uct.n = S.Lct.n = nc;
      S.Uct.nnz = (int64_t)uct_ci.size();
      S.Lct.nnz = (int64_t)lct_ci.size();
      S.Uct.has_diag = true;
    } else {
      S.tUct = TreeSolve();
      S.tLct = TreeSolve();
      build_sweep(S.Uct, nc, uct_cnt, uct_ci, uct_src, &U.v, nullptr, true, true, &udinv, nullptr, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
      build_sweep(S.Lct, nc, lct_cnt, lct_ci, lct_src, &L.v, nullptr, false, false, nullptr, nullptr, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
    }
  } else if (o.coarse_mode == 1) {
    // the Jacobi sweeps of the adjoint run on L~^T and U~^T (the diagonal
    // stays in U~^T's rows; the sweep skips it)
    auto tr = [&](DCsr& T, const DCsr& F) {
      T.n = T.m = nc;
      T.nnz = F.nnz;
      transpose_csr(nc, nc, F.nnz, F.rp.p, F.ci.p, F.v.p, T.rp, T.ci, &T.v, nullptr, s);
    };
    tr(S.dLcT, S.dLc);
    tr(S.dUcT, S.dUc);
  } else if (o.coarse_mode == 2) {
    S.dMcT.n = S.dMcT.m = nc;
    S.dMcT.nnz = S.dMc.nnz;
    transpose_csr(nc, nc, S.dMc.nnz, S.dMc.rp.p, S.dMc.ci.p, S.dMc.v.p, S.dMcT.rp, S.dMcT.ci, &S.dMcT.v, nullptr, s);
  } else {
    S.cinvT.alloc((size_t)S.cnp * S.cnp);
    launch_dense_transpose(nc, S.cnp, S.cinv.p, S.cinvT.p, s);
  }
  if (S.wave) {
    launch_fill_f64_bits(S.wy.p, kSent64, S.wg.total, s);
    launch_fill_f64_bits(S.wt.p, kSent64, S.wg.total, s);
  }
  HIPCK(hipStreamSynchronize(s));
  S.adj_ready = true;
}

// ec = M~_c^{-T} bc, the transpose of the coarse solve (FP64; bc is the
// restriction P^T z, ec holds the sentinel on entry)
static void coarse_adjoint(Solver& S, double* bc, double* ec) {
  hipStream_t s = S.s;
  const int nc = S.nc;
  if (S.opt.coarse_mode == 0 && S.tree_adj) {
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Uct, 8, 8, false));
      launch_tree<double>(S.tUct, bc, false, S.auc.p, nullptr, S.text.p, S.abort_flag.p, s);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Lct, 8, 8, true));
      launch_tree<double>(S.tLct, S.auc.p, false, ec, S.auc.p, S.text.p, S.abort_flag.p, s);
    }
  } else if (S.opt.coarse_mode == 0) {
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Uct, 8, 8, false));
      run_tri<double>(S, S.Uct, bc, false, S.auc.p, nullptr);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, sweep_bytes(S.Lct, 8, 8, true));
      run_tri<double>(S, S.Lct, S.auc.p, false, ec, S.auc.p);
    }
  } else if (S.opt.coarse_mode == 3) {
    Prof p(S, PC_SWEEP_COARSE, (double)nc * nc * 8 + (double)nc * 16);
    launch_dense_gemv<double>(nc, S.cnp, S.cinvT.p, bc, ec, s);
  } else if (S.opt.coarse_mode == 2) {
    Prof p(S, PC_SWEEP_COARSE, (double)S.dMcT.nnz * 12 + (double)nc * 20);
    launch_spmv<double>(nc, S.dMcT.rp.p, S.dMcT.ci.p, S.dMcT.v.p, bc, ec, s);
  } else {
    // the forward sweeps' transpose, factor by factor in reverse order: e <-
    // D^{-1} (bc - (U~^T - D) e) from e = D^{-1} bc, then y <- e - (L~^T - I) y
    // from y = e
    Prof p(S, PC_SWEEP_COARSE, 0.0);
    double* E[2] = {S.auc.p, S.jtmp.p};
    int c = 0;
    launch_jacobi(nc, S.dUcT.rp.p, S.dUcT.ci.p, S.dUcT.v.p, S.ucdinv.p, bc, S.jzero.p, E[0], s);
    for (int k = 0; k < S.opt.coarse_sweeps; ++k) {
      launch_jacobi(nc, S.dUcT.rp.p, S.dUcT.ci.p, S.dUcT.v.p, S.ucdinv.p, bc, E[c], E[1 - c], s);
      c = 1 - c;
    }
    const double* e = E[c];
    double* Y[2] = {ec, E[1 - c]};
    int d = 0;
    d2d(ec, e, nc, s);
    for (int k = 0; k < S.opt.coarse_sweeps; ++k) {
      launch_jacobi(nc, S.dLcT.rp.p, S.dLcT.ci.p, S.dLcT.v.p, nullptr, e, Y[d], Y[1 - d], s);
      d = 1 - d;
    }
    if (Y[d] != ec) d2d(ec, Y[d], nc, s);
  }
}

// t = S^{-T} sv = Q^T L0^{-T} U0^{-T} Q sv (FP64; one column)
static void smooth_adjoint(Solver& S, const double* sv, double* t) {
  hipStream_t s = S.s;
  if (S.wave) {
    Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.U0t, 8, 8, false) + sweep_bytes(S.L0t, 8, 8, true));
    launch_wave_pair<double>(S.wg, S.wU0t, S.wL0t, sv, true, S.wz.p, S.wy.p, S.wt.p, t, S.abort_flag.p, s);
  } else if (S.fine_nd) {
    Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.U0t, 8, 8, false) + sweep_bytes(S.L0t, 8, 8, true) + (double)S.n * 40);
    launch_perm_gather<double>(S.n, S.fperm.p, sv, S.fzp.p, s);
    if (S.ftree_adj) {
      launch_tree<double>(S.tU0t, S.fzp.p, false, S.y.p, nullptr, S.fext.p, S.abort_flag.p, s);
      launch_tree<double>(S.tL0t, S.y.p, false, S.ftp.p, S.y.p, S.fext.p, S.abort_flag.p, s);
    } else {
      run_tri<double>(S, S.U0t, S.fzp.p, false, S.y.p, nullptr);
      run_tri<double>(S, S.L0t, S.y.p, false, S.ftp.p, S.y.p);
    }
    launch_perm_scatter<double>(S.n, S.fperm.p, S.ftp.p, t, s);
  } else {
    {
      Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.U0t, 8, 8, false));
      run_tri<double>(S, S.U0t, sv, false, S.aw.p, nullptr);
    }
    {
      Prof p(S, PC_SWEEP_FINE, sweep_bytes(S.L0t, 8, 8, true));
      run_tri<double>(S, S.L0t, S.aw.p, false, t, S.aw.p);
    }
  }
}

// q = B~^{-T} z (FP64), the transpose of Eq. (twogrid)'s operator:
// ec = M~_c^{-T} P^T z; s = z - A^T P ec; t = S^{-T} s; q = P ec + t
static void vcycle_adjoint(Solver& S, const double* z, double* q) {
  ensure_adjoint(S);
  hipStream_t s = S.s;
  {
    Prof p(S, PC_RESID_RESTRICT, (double)S.n * 12 + (double)S.nc * 16);
    launch_restrict_plain(S.nc, S.aptr.p, S.amem.p, z, S.abc.p, S.aec.p, 0, s);
  }
  coarse_adjoint(S, S.abc.p, S.aec.p);
  {
    Prof p(S, PC_RESID_RESTRICT, (double)S.nnz * 12 + (double)S.n * 24);
    launch_resid_adj(S.n, S.AT.rp.p, S.AT.ci.p, S.AT.v.p, S.agg.p, S.aec.p, z, S.as.p, s);
  }
  smooth_adjoint(S, S.as.p, S.at.p);
  {
    // t is reset to the sentinel only where the level sweeps produce it
    const bool reset_t = !S.wave && !S.fine_nd;
    Prof p(S, PC_PROLONG, (double)S.n * 28 + (double)S.nc * 8);
    launch_prolong<double>(S.n, S.agg.p, S.at.p, S.aec.p, q, 0, s, reset_t);
  }
}

static void apply_op(Solver& S, bool adjoint, const double* x, double* y) {
  Prof p(S, PC_SPMV, (double)S.nnz * 12 + (double)S.n * 20);
  const DCsr& M = adjoint ? S.AT : S.A;
  launch_spmv<double>(S.n, M.rp.p, M.ci.p, M.v.p, x, y, S.s, S.spmv_cap);
}

static void ensure_krylov(Solver& S, int m) {
  if (m <= S.mcap && S.V.p) return;
  S.mcap = m;
  // basis vectors are ld doubles apart: n rounded up to 64, plus an odd
  // multiple of 512 bytes, so that the many-vector passes' concurrent
  // segments of different vectors do not all fall on the same HBM channels
  // (a power-of-two stride did: 596 -> 541 us per step on 1024^2)
  S.ld = ((size_t)S.n + 63) / 64 * 64 + (size_t)64 * 29;
  S.V.alloc(S.ld * (m + 1));
  S.Z.alloc(S.ld * m);
  S.w.alloc(S.ld);
  S.coef.alloc(kMaxRestart + 8);
  S.ldg = (size_t)m + 1;
  S.gram.alloc(S.ldg * S.ldg);
  S.gcoef.alloc((size_t)m + 8);
  S.gdots.alloc((size_t)m + 8);
}

// ------------------------------------------------------------------ FGMRES
struct OneResult {
  gmg_status st;
  int steps, restarts;
  double relres, est;
};

// Flexible GMRES(m) with right preconditioning (Algorithm 1's accelerator with
// z_j = B~^{-1} v_j kept), Givens rotations on the host (O(m) scalars per
// step).  Orthogonalisation: classical Gram-Schmidt applied twice while the
// basis is short (up to 32 vectors); beyond, one projection whose coefficients
// are corrected with the basis' Gram matrix G = V^T V, c = (2I - G) V^T w
// (equal to the second pass's V^T (w - V h) = h - G h), where each new row of
// G comes from the products V^T w_new taken in the same read of V that forms
// w_new: two reads of V per step instead of three.
static OneResult fgmres(Solver& S, bool adjoint, int precision, const double* b, double* x, double tol,
                        int maxit, int m, bool x0_given) {
  hipStream_t s = S.s;
  const int64_t n = S.n;
  ensure_krylov(S, m);
  const size_t ld = S.ld;
  double* V = S.V.p;
  double* Z = S.Z.p;
  double* w = S.w.p;
  double* res = S.rw.result.p;
  double* hp = S.hpin;
  OneResult out{GMG_NOT_CONVERGED, 0, 0, 0.0, 0.0};
  if (!x0_given) HIPCK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  {
    Prof p(S, PC_VECTOR, (double)n * 8);
    launch_norm2(b, n, S.rw, res, s);
  }
  d2h(hp, res, 1, s);
  HIPCK(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(hp[0]);
  if (!std::isfinite(bnorm)) { out.st = GMG_ERR_NONFINITE; return out; }
  if (bnorm == 0.0) {
    HIPCK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    HIPCK(hipStreamSynchronize(s));
    out.st = GMG_OK;
    return out;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m + 1), sn(m + 1), g(m + 2), yv(m + 1);
  auto HH = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  int total = 0;
  double rate = 1.0;   // last ratio of successive residual estimates
  for (;;) {
    {
      Prof p(S, PC_SPMV, (double)S.nnz * 12 + (double)n * 28);
      const DCsr& M = adjoint ? S.AT : S.A;
      launch_residual(S.n, M.rp.p, M.ci.p, M.v.p, x, b, w, s, S.spmv_cap);
    }
    {
      Prof p(S, PC_VECTOR, (double)n * 8);
      launch_norm2(w, n, S.rw, res, s);
    }
    d2h(hp, res, 1, s);
    HIPCK(hipStreamSynchronize(s));
    const double beta = std::sqrt(hp[0]);
    out.relres = beta / bnorm;
    if (!std::isfinite(out.relres)) { out.st = GMG_ERR_NONFINITE; break; }
    if (out.relres < tol) { out.st = GMG_OK; break; }
    if (total >= maxit) { out.st = GMG_NOT_CONVERGED; break; }
    if (total > 0) ++out.restarts;
    {
      Prof p(S, PC_VECTOR, (double)n * 16);
      launch_scale(w, 1.0 / beta, V, n, s);
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // Steps run one deep in a pipeline: the host reads step j's Hessenberg
    // column (Givens rotation, convergence test) while the GPU already runs
    // step j + 1, whose basis vector the GPU normalises itself.  A step
    // enqueued after the last one needed is left unused: the update below
    // takes only Z's first k columns, so iterates and step counts are those
    // of the plain loop.
    int k = 0;
    bool breakdown = false;
    auto enqueue_step = [&](int j) {
      double* vj = V + (size_t)j * ld;
      double* zj = Z + (size_t)j * ld;
      if (adjoint) vcycle_adjoint(S, vj, zj);
      else if (precision == 1) vcycle<float>(S, vj, zj);
      else vcycle<double>(S, vj, zj);
      apply_op(S, adjoint, zj, w);
      const int kc = j + 1;
      // classical Gram-Schmidt, twice: h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2
      double* h1 = res;
      double* h2 = res + kc;
      double* nrm = res + 2 * kc;
      const double* gdots = nullptr;  // V^T w_new when the pass took them (a Gram row), else the row is zero
      const double* nrm_src = nrm;
      if (kc <= kFused) {
        Prof p(S, PC_ORTHO, 8.0 * n * (3 * kc + 6));
        launch_multidot(V, ld, kc, w, n, S.rw, h1, s);
        launch_update_dot(V, ld, kc, h1, w, n, S.rw, h2, s);
        launch_update_norm(V, ld, kc, h2, w, n, S.rw, nrm, s);
      } else if (kc <= many_max()) {
        // h1 = V^T w; c = (2I - G) h1 (its correction d = c - h1 into h2's
        // slot, where the host adds it); w <- w - V c with V^T w and ||w||^2
        // in the same read of V
        Prof p(S, PC_ORTHO, 8.0 * n * (2 * kc + 3) + 8.0 * kc * kc);
        launch_multidot_many(V, ld, kc, w, n, S.rw, h1, s);
        launch_gram_coef(kc, h1, S.gram.p, S.ldg, h2, S.gcoef.p, s);
        launch_update_dot_many(V, ld, kc, S.gcoef.p, w, n, true, S.rw, S.gdots.p, s);
        gdots = S.gdots.p;
        nrm_src = S.gdots.p + kc;
      } else {
        // the same projection over blocks of mm vectors: h1 block by block;
        // w -= V_b c_b for all blocks but the last, whose pass also takes its
        // products with w_new and ||w_new||^2; then the other blocks'
        // products with w_new (the Gram row)
        const int mm = many_max(), nb = (kc + mm - 1) / mm, kl = kc - mm * (nb - 1);
        Prof p(S, PC_ORTHO, 8.0 * n * (3 * kc - kl + 4 * nb) + 8.0 * kc * kc);
        for (int b = 0; b < nb; ++b)
          launch_multidot_many(V + (size_t)b * mm * ld, ld, std::min(mm, kc - b * mm), w, n, S.rw, h1 + b * mm, s);
        launch_gram_coef(kc, h1, S.gram.p, S.ldg, h2, S.gcoef.p, s);
        for (int b = 0; b + 1 < nb; ++b)
          launch_update_many(V + (size_t)b * mm * ld, ld, mm, S.gcoef.p + b * mm, w, n, false, S.rw, nullptr, s);
        const int b0 = mm * (nb - 1);
        launch_update_dot_many(V + (size_t)b0 * ld, ld, kl, S.gcoef.p + b0, w, n, true, S.rw, S.gdots.p + b0, s);
        for (int b = 0; b + 1 < nb; ++b)
          launch_multidot_many(V + (size_t)b * mm * ld, ld, mm, w, n, S.rw, S.gdots.p + b * mm, s);
        gdots = S.gdots.p;
        nrm_src = S.gdots.p + kc;
      }
      {
        Prof p(S, PC_VECTOR, (double)n * 16);
        launch_normalize_gram(w, nrm_src, V + (size_t)(j + 1) * ld, n, j + 1, gdots, S.gram.p, S.ldg,
                              nrm_src == nrm ? nullptr : nrm, s);
      }
      d2h(hp + (size_t)kPinCol * (1 + (j & 1)), res, 2 * kc + 1, s);
      HIPCK(hipEventRecord(S.colev[j & 1], s));
    };
    // true when the cycle ends with step j
    auto process_step = [&](int j) -> bool {
      HIPCK(hipEventSynchronize(S.colev[j & 1]));
      const double* col = hp + (size_t)kPinCol * (1 + (j & 1));
      const int kc = j + 1;
      for (int i = 0; i <= j; ++i) HH(i, j) = col[i] + col[kc + i];
      const double hn = std::sqrt(col[2 * kc]);
      HH(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const double a = HH(i, j), c = HH(i + 1, j);
        HH(i, j) = cs[i] * a + sn[i] * c;
        HH(i + 1, j) = -sn[i] * a + cs[i] * c;
      }
      const double rho = std::hypot(HH(j, j), HH(j + 1, j));
      if (rho == 0.0 || !std::isfinite(rho)) {
        out.st = std::isfinite(rho) ? GMG_ERR_BREAKDOWN : GMG_ERR_NONFINITE;
        breakdown = true;
        return true;
      }
      cs[j] = HH(j, j) / rho;
      sn[j] = HH(j + 1, j) / rho;
      HH(j, j) = rho;
      HH(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      k = j + 1;
      const double prev = out.est;
      out.est = std::fabs(g[j + 1]) / bnorm;
      if (prev > 0.0 && j > 0) rate = out.est / prev;
      S.hist.push_back(out.est);
      if (S.log_every > 0 && total % S.log_every == 0) {
        std::fprintf(stderr, "[gmg] step %d  estimated relres %.3e\n", total, out.est);
        std::fflush(stderr);
      }
      return out.est < tol || hn == 0.0 || total >= maxit;
    };
    // Near the end of a cycle (the next step reaches maxit, or at the recent
    // rate of decrease it reaches tol) step j - 1 is processed before step j
    // is enqueued, so no step past the last one needed is launched.
    bool ended = false;
    for (int j = 0; j < m && !ended; ++j) {
      const bool near_end =
          j > 0 && (total + 1 >= maxit || (out.est > 0.0 && out.est * std::min(rate, 1.0) < 2.0 * tol));
      if (near_end) {
        ended = process_step(j - 1);
        if (ended) break;
        enqueue_step(j);
      } else {
        enqueue_step(j);
        if (j > 0) ended = process_step(j - 1);
      }
    }
    if (!ended) process_step(m - 1);
    check_abort(S);
    if (breakdown) break;
    for (int i = k - 1; i >= 0; --i) {
      double sum = g[i];
      for (int l = i + 1; l < k; ++l) sum -= HH(i, l) * yv[l];
      yv[i] = sum / HH(i, i);
    }
    h2d(S.coef.p, yv.data(), k, s);
    {
      Prof p(S, PC_VECTOR, 8.0 * n * (k + 2));
      launch_xupdate(x, Z, ld, k, S.coef.p, n, s);
    }
  }
  out.steps = total;
  // a reduction that gave up on a partial (its bounded wait ran out) may see
  // that partial land later: start the next solve from clean partials
  if (out.st == GMG_ERR_NONFINITE || out.st == GMG_ERR_BREAKDOWN) red_reset(S.rw, s);
  HIPCK(hipStreamSynchronize(s));
  return out;
}

// ------------------------------------------------------- multi-RHS solve
// Several right-hand sides share every launch: the fine wavefront sweeps and
// the coarse tree solves run all columns in one launch (a column's
// dependency chains interleave with the others', so the latency-bound sweeps
// cost about what one column costs), the matrix, the aggregates and the
// factors are read once per step for all columns, and the Krylov kernels run
// one recurrence per column of their grid.
constexpr int kBatchRS = 2 * kFused + 8;  // result doubles per column: h1, h2, ||w||^2

static void ensure_batch(Solver& S, int nb, int m, bool f32, bool adjoint) {
  BatchWork& B = S.bw;
  hipStream_t s = S.s;
  const bool grow = nb > B.cap || m > B.m;
  if (grow) {
    B = BatchWork();
    B.cap = BATCH_MAX;
    B.m = std::max(m, kFused);
    B.ld = ((size_t)S.n + 63) / 64 * 64;
    B.ldc = ((size_t)std::max(S.nc, 1) + 63) / 64 * 64;
    const size_t nf = B.ld * B.cap, ncv = B.ldc * B.cap;
    B.t.alloc(nf);
    B.r.alloc(nf);
    B.rc.alloc(ncv);
    B.yc.alloc(ncv);
    B.ec.alloc(ncv);
    B.text.alloc(ncv);
    launch_fill_f64_bits(B.t.p, kSent64, nf, s);
    launch_fill_f64_bits(B.yc.p, kSent64, ncv, s);
    launch_fill_f64_bits(B.ec.p, kSent64, ncv, s);
    launch_fill_f64_bits(B.text.p, kSent64, ncv, s);
    if (S.wave) {
      const size_t nw = (size_t)S.wg.total * B.cap;
      B.wz.alloc(nw);
      B.wy.alloc(nw);
      B.wt.alloc(nw);
      launch_fill_f64_bits(B.wy.p, kSent64, nw, s);
      launch_fill_f64_bits(B.wt.p, kSent64, nw, s);
    }
    auto counters = [&](DBuf<int>& c, const TreeSolve& t) {
      if (!t.ncount.p) return;
      c.alloc(t.ncount.n * B.cap);
      launch_fill_u32(reinterpret_cast<unsigned*>(c.p), 0u, c.n, s);
    };
    counters(B.ncLc, S.tLc);
    counters(B.ncUc, S.tUc);
    B.V.alloc(B.ld * B.cap * (B.m + 1));
    B.Z.alloc(B.ld * B.cap * B.m);
    B.w.alloc(nf);
    B.x.alloc(nf);
    B.b.alloc(nf);
    B.coef.alloc((size_t)B.cap * (B.m + 1));
  }
  if (f32 && !B.f32) {
    const size_t nf = B.ld * B.cap, ncv = B.ldc * B.cap;
    B.t32.alloc(nf);
    B.r32.alloc(nf);
    B.rc32.alloc(ncv);
    B.yc32.alloc(ncv);
    B.ec32.alloc(ncv);
    B.text32.alloc(ncv);
    launch_fill_f32_bits(B.t32.p, kSent32, nf, s);
    launch_fill_f32_bits(B.yc32.p, kSent32, ncv, s);
    launch_fill_f32_bits(B.ec32.p, kSent32, ncv, s);
    launch_fill_f32_bits(B.text32.p, kSent32, ncv, s);
    if (S.wave) {
      const size_t nw = (size_t)S.wg.total * B.cap;
      B.wz32.alloc(nw);
      B.wy32.alloc(nw);
      B.wt32.alloc(nw);
      launch_fill_f32_bits(B.wy32.p, kSent32, nw, s);
      launch_fill_f32_bits(B.wt32.p, kSent32, nw, s);
    }
    B.f32 = true;
  }
  if (adjoint && !B.adj) {
    const size_t nf = B.ld * B.cap, ncv = B.ldc * B.cap;
    B.abc.alloc(ncv);
    B.auc.alloc(ncv);
    B.aec.alloc(ncv);
    B.as.alloc(nf);
    B.at.alloc(nf);
    launch_fill_f64_bits(B.auc.p, kSent64, ncv, s);
    launch_fill_f64_bits(B.aec.p, kSent64, ncv, s);
    launch_fill_f64_bits(B.at.p, kSent64, nf, s);
    auto counters = [&](DBuf<int>& c, const TreeSolve& t) {
      if (!t.ncount.p) return;
      c.alloc(t.ncount.n * B.cap);
      launch_fill_u32(reinterpret_cast<unsigned*>(c.p), 0u, c.n, s);
    };
    counters(B.ncUct, S.tUct);
    counters(B.ncLct, S.tLct);
    B.adj = true;
  }
}

// Every value-as-flag buffer of the batch back to its idle state (sentinels,
// zero node counters), so a solve never inherits state from one that stopped
// early.
static void reset_batch_buffers(Solver& S) {
  BatchWork& B = S.bw;
  hipStream_t s = S.s;
  for (DBuf<double>* b : {&B.t, &B.yc, &B.ec, &B.text, &B.wy, &B.wt, &B.auc, &B.aec, &B.at})
    if (b->p) launch_fill_f64_bits(b->p, kSent64, b->n, s);
  for (DBuf<float>* b : {&B.t32, &B.yc32, &B.ec32, &B.text32, &B.wy32, &B.wt32})
    if (b->p) launch_fill_f32_bits(b->p, kSent32, b->n, s);
  for (DBuf<int>* c : {&B.ncLc, &B.ncUc, &B.ncUct, &B.ncLct})
    if (c->p) launch_fill_u32(reinterpret_cast<unsigned*>(c->p), 0u, c->n, s);
}

// q_c = B~^{-1} z_c for the columns c < nb (z_c = z + c * ldz, q_c = q + c * ldq)
template <class T>
static void vcycle_batch(Solver& S, const double* z, size_t ldz, double* q, size_t ldq, int nb) {
  constexpr bool F32 = sizeof(T) == 4;
  BatchWork& B = S.bw;
  hipStream_t s = S.s;
  T* t = F32 ? (T*)B.t32.p : (T*)B.t.p;
  T* rc = F32 ? (T*)B.rc32.p : (T*)B.rc.p;
  T* yc = F32 ? (T*)B.yc32.p : (T*)B.yc.p;
  T* ec = F32 ? (T*)B.ec32.p : (T*)B.ec.p;
  const T* Av = F32 ? (const T*)S.A.v32.p : (const T*)S.A.v.p;
  const size_t sz = sizeof(T), ld = B.ld, ldc = B.ldc;
  if (S.wave) {
    Prof p(S, PC_SWEEP_FINE, nb * (sweep_bytes(S.L0, sz, 8, false) + sweep_bytes(S.U0, sz, sz, true)));
    launch_wave_pair<T>(S.wg, S.wL0, S.wU0, z, true, F32 ? (T*)B.wz32.p : (T*)B.wz.p, F32 ? (T*)B.wy32.p : (T*)B.wy.p,
                        F32 ? (T*)B.wt32.p : (T*)B.wt.p, t, S.abort_flag.p, s, nb, ldz, ld);
  } else {
    for (int c = 0; c < nb; ++c) smooth_apply<T>(S, z + c * ldz, t + c * ld);
  }
  {
    // the residual over the column batch (A read once for every column),
    // then the restriction; measured faster than one kernel that sums each
    // aggregate's members' residuals itself (gathers by member are not
    // coalesced: 306 us against 81 us for 16 columns on 512^2)
    Prof p(S, PC_RESID_RESTRICT, (double)S.nnz * (4 + sz) + (double)S.n * 8 +
                                     nb * ((double)S.n * (8 + 3 * sz + 4) + (double)S.nc * 2 * sz));
    T* r = F32 ? (T*)B.r32.p : (T*)B.r.p;
    launch_resid_fine_cols<T>(S.n, S.A.rp.p, S.A.ci.p, Av, t, ld, z, ldz, r, ld, nb, s);
    launch_restrict_cols_t<T>(S.nc, S.aptr.p, S.amem.p, r, ld, rc, ec, ldc, nb, s);
  }
  if (S.opt.coarse_mode == 0 && S.tree) {
    T* ext = F32 ? (T*)B.text32.p : (T*)B.text.p;
    {
      Prof p(S, PC_SWEEP_COARSE, nb * sweep_bytes(S.Lc, sz, sz, false));
      launch_tree<T>(S.tLc, rc, false, yc, nullptr, ext, S.abort_flag.p, s, nb, ldc, B.ncLc.p);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, nb * sweep_bytes(S.Uc, sz, sz, true));
      launch_tree<T>(S.tUc, yc, false, ec, yc, ext, S.abort_flag.p, s, nb, ldc, B.ncUc.p);
    }
  } else {
    for (int c = 0; c < nb; ++c) coarse_apply<T>(S, rc + c * ldc, ec + c * ldc);
  }
  {
    Prof p(S, PC_PROLONG, nb * ((double)S.n * (4 + 2 * sz + 8) + (double)S.nc * sz));
    launch_prolong_cols<T>(S.n, S.agg.p, t, ld, ec, ldc, q, ldq, nb, s);
  }
}

// q_c = B~^{-T} z_c (FP64) for the columns c < nb
static void vcycle_adjoint_batch(Solver& S, const double* z, size_t ldz, double* q, size_t ldq, int nb) {
  ensure_adjoint(S);
  ensure_batch(S, nb, S.bw.m, false, true);
  BatchWork& B = S.bw;
  hipStream_t s = S.s;
  const size_t ld = B.ld, ldc = B.ldc;
  {
    Prof p(S, PC_RESID_RESTRICT, nb * ((double)S.n * 12 + (double)S.nc * 16));
    launch_restrict_cols(S.nc, S.aptr.p, S.amem.p, z, ldz, B.abc.p, B.aec.p, ldc, nb, s);
  }
  if (S.opt.coarse_mode == 0 && S.tree_adj) {
    {
      Prof p(S, PC_SWEEP_COARSE, nb * sweep_bytes(S.Uct, 8, 8, false));
      launch_tree<double>(S.tUct, B.abc.p, false, B.auc.p, nullptr, B.text.p, S.abort_flag.p, s, nb, ldc, B.ncUct.p);
    }
    {
      Prof p(S, PC_SWEEP_COARSE, nb * sweep_bytes(S.Lct, 8, 8, true));
      launch_tree<double>(S.tLct, B.auc.p, false, B.aec.p, B.auc.p, B.text.p, S.abort_flag.p, s, nb, ldc, B.ncLct.p);
    }
  } else {
    for (int c = 0; c < nb; ++c) coarse_adjoint(S, B.abc.p + c * ldc, B.aec.p + c * ldc);
  }
  {
    Prof p(S, PC_RESID_RESTRICT, (double)S.nnz * 12 + (double)S.n * 4 + nb * ((double)S.n * 24 + (double)S.nc * 8));
    launch_resid_adj_cols(S.n, S.AT.rp.p, S.AT.ci.p, S.AT.v.p, S.agg.p, B.aec.p, ldc, z, ldz, B.as.p, ld, nb, s);
  }
  if (S.wave) {
    Prof p(S, PC_SWEEP_FINE, nb * (sweep_bytes(S.U0t, 8, 8, false) + sweep_bytes(S.L0t, 8, 8, true)));
    launch_wave_pair<double>(S.wg, S.wU0t, S.wL0t, B.as.p, true, B.wz.p, B.wy.p, B.wt.p, B.at.p, S.abort_flag.p, s, nb,
                             ld, ld);
  } else {
    for (int c = 0; c < nb; ++c) smooth_adjoint(S, B.as.p + c * ld, B.at.p + c * ld);
  }
  {
    Prof p(S, PC_PROLONG, nb * ((double)S.n * 28 + (double)S.nc * 8));
    launch_prolong_cols<double>(S.n, S.agg.p, B.at.p, ld, B.aec.p, ldc, q, ldq, nb, s);
  }
}

struct BatchResult {
  gmg_status st = GMG_OK;
  int steps = 0, restarts = 0, converged = 0;
  double relres = 0.0, est = 0.0;
};

// FGMRES(m), m <= 32, on nb columns at once (columns c0 .. c0 + nb - 1 of the
// caller's (N, nrhs) arrays): one recurrence per column, every launch shared.
// Each column keeps its own Hessenberg matrix, rotations and step count; a
// column that has converged is carried along (its further steps are not
// used) until the cycle ends, then left out of the restarts.
static BatchResult fgmres_batch(Solver& S, bool adjoint, int precision, const double* Bu, double* Xu, int nrhs,
                                int c0, int nb, double tol, int maxit, int m, bool x0_given) {
  hipStream_t s = S.s;
  const int64_t n = S.n;
  if (adjoint) ensure_adjoint(S);   // the transposed factors, before their per-column counters
  ensure_batch(S, nb, m, precision == 1, adjoint);
  reset_batch_buffers(S);
  BatchWork& W = S.bw;
  const size_t ld = W.ld, cap = (size_t)W.cap;
  double* res = S.rw.result.p;
  double* hp = S.hpin;
  BatchResult out;
  const BatchCols bcol{nb, ld, ld, (size_t)kBatchRS, (size_t)kBatchRS};
  const DCsr& M = adjoint ? S.AT : S.A;
  launch_cols_from_rows(Bu, nrhs, c0, W.b.p, ld, n, nb, s);
  if (x0_given) launch_cols_from_rows(Xu, nrhs, c0, W.x.p, ld, n, nb, s);
  else HIPCK(hipMemsetAsync(W.x.p, 0, sizeof(double) * ld * nb, s));
  {
    Prof p(S, PC_VECTOR, (double)n * 8 * nb);
    launch_norm2(W.b.p, n, S.rw, res, s, nb, ld, 1);
  }
  d2h(hp, res, nb, s);
  HIPCK(hipStreamSynchronize(s));
  std::vector<double> bnorm(nb);
  for (int c = 0; c < nb; ++c) {
    bnorm[c] = std::sqrt(hp[c]);
    if (!std::isfinite(bnorm[c])) { out.st = GMG_ERR_NONFINITE; return out; }
  }
  const int mm = m + 1;
  std::vector<double> H((size_t)nb * mm * m, 0.0), cs((size_t)nb * mm), sn((size_t)nb * mm), g((size_t)nb * (m + 2)),
      yv((size_t)nb * mm), coef((size_t)cap * mm, 0.0), relres(nb, 0.0), est(nb, 0.0);
  auto HH = [&](int c, int i, int j) -> double& { return H[((size_t)c * mm + i) * m + j]; };
  std::vector<int> total(nb, 0), kc_used(nb, 0), restarts(nb, 0);
  std::vector<char> done(nb, 0), live(nb, 0);
  std::vector<std::vector<double>> hist(nb);
  for (int c = 0; c < nb; ++c)
    if (bnorm[c] == 0.0) done[c] = 1;   // x = 0 (set below) is exact
  for (;;) {
    // r_c = b_c - A x_c and its norm, every column
    {
      Prof p(S, PC_SPMV, (double)S.nnz * 12 + (double)n * 4 + (double)n * 20 * nb);
      launch_residual_cols((int)n, M.rp.p, M.ci.p, M.v.p, W.x.p, ld, W.b.p, ld, W.w.p, ld, nb, s);
    }
    {
      Prof p(S, PC_VECTOR, (double)n * 8 * nb);
      launch_norm2(W.w.p, n, S.rw, res, s, nb, ld, 1);
    }
    d2h(hp, res, nb, s);
    HIPCK(hipStreamSynchronize(s));
    bool any = false;
    for (int c = 0; c < nb; ++c) {
      if (done[c] && bnorm[c] == 0.0) { relres[c] = 0.0; continue; }
      const double beta = std::sqrt(hp[c]);
      relres[c] = beta / bnorm[c];
      live[c] = 0;
      if (!std::isfinite(relres[c])) { out.st = GMG_ERR_NONFINITE; red_reset(S.rw, s); return out; }
      if (relres[c] < tol) { done[c] = 1; continue; }
      if (total[c] >= maxit) { done[c] = 1; continue; }
      if (total[c] > 0) ++restarts[c];
      live[c] = 1;
      any = true;
      std::fill(&g[(size_t)c * (m + 2)], &g[(size_t)c * (m + 2)] + (m + 2), 0.0);
      g[(size_t)c * (m + 2)] = beta;
      kc_used[c] = 0;
    }
    if (!any) break;
    // v_1 = r / ||r|| for every column (finished ones carried along)
    {
      Prof p(S, PC_VECTOR, (double)n * 16 * nb);
      launch_normalize_cols(W.w.p, ld, res, 1, W.V.p, ld, n, nb, s);
    }
    bool breakdown = false;
    auto enqueue_step = [&](int j) {
      double* vj = W.V.p + (size_t)j * cap * ld;
      double* zj = W.Z.p + (size_t)j * cap * ld;
      if (adjoint) vcycle_adjoint_batch(S, vj, ld, zj, ld, nb);
      else if (precision == 1) vcycle_batch<float>(S, vj, ld, zj, ld, nb);
      else vcycle_batch<double>(S, vj, ld, zj, ld, nb);
      {
        Prof p(S, PC_SPMV, (double)S.nnz * 12 + (double)n * 4 + (double)n * 16 * nb);
        launch_spmm<double>((int)n, M.rp.p, M.ci.p, M.v.p, zj, ld, W.w.p, ld, nb, s);
      }
      const int kc = j + 1;
      {
        // classical Gram-Schmidt twice, every column in each launch
        Prof p(S, PC_ORTHO, 8.0 * n * (3 * kc + 6) * nb);
        launch_multidot(W.V.p, cap * ld, kc, W.w.p, n, S.rw, res, s, bcol);
        launch_update_dot(W.V.p, cap * ld, kc, res, W.w.p, n, S.rw, res + kc, s, bcol);
        launch_update_norm(W.V.p, cap * ld, kc, res + kc, W.w.p, n, S.rw, res + 2 * kc, s, bcol);
      }
      {
        Prof p(S, PC_VECTOR, (double)n * 16 * nb);
        launch_normalize_cols(W.w.p, ld, res + 2 * kc, kBatchRS, W.V.p + (size_t)(j + 1) * cap * ld, ld, n, nb, s);
      }
      d2h(hp + (size_t)kPinCol * (1 + (j & 1)), res, (size_t)nb * kBatchRS, s);
      HIPCK(hipEventRecord(S.colev[j & 1], s));
    };
    // true when every column's cycle has ended with step j
    auto process_step = [&](int j) -> bool {
      HIPCK(hipEventSynchronize(S.colev[j & 1]));
      const int kc = j + 1;
      bool all_ended = true;
      for (int c = 0; c < nb; ++c) {
        if (!live[c]) continue;
        const double* col = hp + (size_t)kPinCol * (1 + (j & 1)) + (size_t)c * kBatchRS;
        double* gc = &g[(size_t)c * (m + 2)];
        double* csc = &cs[(size_t)c * mm];
        double* snc = &sn[(size_t)c * mm];
        for (int i = 0; i <= j; ++i) HH(c, i, j) = col[i] + col[kc + i];
        const double hn = std::sqrt(col[2 * kc]);
        HH(c, j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
          const double a = HH(c, i, j), b2 = HH(c, i + 1, j);
          HH(c, i, j) = csc[i] * a + snc[i] * b2;
          HH(c, i + 1, j) = -snc[i] * a + csc[i] * b2;
        }
        const double rho = std::hypot(HH(c, j, j), HH(c, j + 1, j));
        if (rho == 0.0 || !std::isfinite(rho)) {
          out.st = std::isfinite(rho) ? GMG_ERR_BREAKDOWN : GMG_ERR_NONFINITE;
          breakdown = true;
          return true;
        }
        csc[j] = HH(c, j, j) / rho;
        snc[j] = HH(c, j + 1, j) / rho;
        HH(c, j, j) = rho;
        HH(c, j + 1, j) = 0.0;
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        ++total[c];
        kc_used[c] = j + 1;
        est[c] = std::fabs(gc[j + 1]) / bnorm[c];
        hist[c].push_back(est[c]);
        if (est[c] < tol || hn == 0.0 || total[c] >= maxit) live[c] = 0;
        else all_ended = false;
      }
      return all_ended;
    };
    std::vector<char> in_cycle(live);
    bool ended = false;
    for (int j = 0; j < m && !ended; ++j) {
      enqueue_step(j);
      if (j > 0) ended = process_step(j - 1);
    }
    if (!ended) process_step(m - 1);
    check_abort(S);
    if (breakdown) { red_reset(S.rw, s); break; }
    // x_c += Z_c y_c with each column's own step count (zeros for the others)
    int kmax = 0;
    std::fill(coef.begin(), coef.end(), 0.0);
    for (int c = 0; c < nb; ++c) {
      if (!in_cycle[c]) continue;
      const int k = kc_used[c];
      kmax = std::max(kmax, k);
      double* y = &yv[(size_t)c * mm];
      const double* gc = &g[(size_t)c * (m + 2)];
      for (int i = k - 1; i >= 0; --i) {
        double sum = gc[i];
        for (int l = i + 1; l < k; ++l) sum -= HH(c, i, l) * y[l];
        y[i] = sum / HH(c, i, i);
      }
      for (int i = 0; i < k; ++i) coef[(size_t)c * mm + i] = y[i];
      live[c] = 0;
    }
    if (kmax > 0) {
      h2d(W.coef.p, coef.data(), (size_t)nb * mm, s);
      Prof p(S, PC_VECTOR, 8.0 * n * (kmax + 2) * nb);
      launch_xupdate(W.x.p, W.Z.p, cap * ld, kmax, W.coef.p, n, s, nb, ld, ld, (size_t)mm);
    }
  }
  for (int c = 0; c < nb; ++c)
    if (bnorm[c] == 0.0) HIPCK(hipMemsetAsync(W.x.p + (size_t)c * ld, 0, sizeof(double) * n, s));
  launch_rows_from_cols(Xu, nrhs, c0, W.x.p, ld, n, nb, s);
  HIPCK(hipStreamSynchronize(s));
  for (int c = 0; c < nb; ++c) {
    S.hist.insert(S.hist.end(), hist[c].begin(), hist[c].end());
    out.steps += total[c];
    out.restarts += restarts[c];
    out.relres = std::max(out.relres, relres[c]);
    out.est = std::max(out.est, est[c]);
    if (relres[c] < tol || bnorm[c] == 0.0) ++out.converged;
  }
  if (out.st == GMG_OK && out.converged < nb) out.st = GMG_NOT_CONVERGED;
  return out;
}

static gmg_status solve_impl(Solver& S, bool adjoint, const double* b, double* x, int nrhs, double tol,
                             const gmg_options* o, gmg_info* info) {
  if (!b || !x || nrhs < 1) fail(GMG_ERR_INVALID_ARG, "solve: null vector or nrhs < 1");
  if (!(tol >= 0.0)) fail(GMG_ERR_INVALID_ARG, "solve: tol must be >= 0");
  gmg_options opt = S.opt;
  if (o) {
    opt.x0_given = o->x0_given;
    opt.maxit = o->maxit;
    opt.restart = o->restart;
    opt.precond_fp32 = o->precond_fp32;
  }
  if (opt.restart < 1 || opt.restart > kMaxRestart) fail(GMG_ERR_INVALID_ARG, "restart must be in [1, 2048]");
  if (opt.maxit < 0) fail(GMG_ERR_INVALID_ARG, "maxit must be >= 0");
  if (adjoint && opt.precond_fp32) fail(GMG_ERR_INVALID_ARG, "the adjoint solve runs in FP64 (precond_fp32 0)");
  auto t0 = std::chrono::steady_clock::now();
  reset_cycle_buffers(S);
  S.hist.clear();
  gmg_status worst = GMG_OK;
  int iters = 0, restarts = 0, conv = 0;
  double rel = 0.0, est = 0.0;
  // several right-hand sides with a short restart (the register-resident
  // Krylov kernels) share every launch, in batches of BATCH_MAX columns;
  // otherwise the columns are solved one after another
  const bool batched = nrhs > 1 && opt.restart <= kFused && !S.force_column_loop;
  if (batched) {
    for (int c0 = 0; c0 < nrhs; c0 += BATCH_MAX) {
      const int nb = std::min(BATCH_MAX, nrhs - c0);
      BatchResult r = fgmres_batch(S, adjoint, opt.precond_fp32 ? 1 : 0, b, x, nrhs, c0, nb, tol, opt.maxit,
                                   opt.restart, opt.x0_given != 0);
      iters += r.steps;
      restarts += r.restarts;
      conv += r.converged;
      rel = std::max(rel, r.relres);
      est = std::max(est, r.est);
      if (r.st < 0) { worst = r.st; break; }
      if (r.st > 0 && worst == GMG_OK) worst = r.st;
    }
  } else {
    ensure_krylov(S, opt.restart);
    if (nrhs > 1 && !S.xcol.p) {
      S.xcol.alloc(S.n);
      S.bcol.alloc(S.n);
    }
    for (int c = 0; c < nrhs; ++c) {
      const double* bc = b;
      double* xc = x;
      if (nrhs > 1) {
        launch_get_col(b, nrhs, c, S.bcol.p, S.n, S.s);
        if (opt.x0_given) launch_get_col(x, nrhs, c, S.xcol.p, S.n, S.s);
        bc = S.bcol.p;
        xc = S.xcol.p;
      }
      OneResult r = fgmres(S, adjoint, opt.precond_fp32 ? 1 : 0, bc, xc, tol, opt.maxit, opt.restart,
                           opt.x0_given != 0);
      if (nrhs > 1) launch_set_col(x, nrhs, c, S.xcol.p, S.n, S.s);
      iters += r.steps;
      restarts += r.restarts;
      rel = std::max(rel, r.relres);
      est = std::max(est, r.est);
      if (r.st == GMG_OK) ++conv;
      if (r.st < 0) { worst = r.st; break; }
      if (r.st > 0 && worst == GMG_OK) worst = r.st;
    }
  }
  HIPCK(hipStreamSynchronize(S.s));
  auto t1 = std::chrono::steady_clock::now();
  S.info.iters = iters;
  S.info.restarts = restarts;
  S.info.converged = conv;
  S.info.relres_true = rel;
  S.info.relres_est = est;
  S.info.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (info) *info = S.info;
  if (worst == GMG_ERR_BREAKDOWN) fail(worst, "FGMRES breakdown (zero Givens column)");
  if (worst == GMG_ERR_NONFINITE) fail(worst, "non-finite residual");
  return worst;
}

// ------------------------------------------------------------------- setup
static std::vector<int> to_host_int(const int* d, size_t n, hipStream_t s) {
  std::vector<int> h(n);
  d2h_large(h.data(), d, n, s);
  return h;
}

// 2D-grid structure of a triangular factor given by dependency lists: every
// dependency of row k is k -/+ 1 (same grid row) or k -/+ nx, for one nx
// dividing n (lower: minus, upper: plus).  Returns nx, or 0.
static int grid2d_nx(int n, const std::vector<int>& dep_rp, const std::vector<int>& dep_ci, bool lower) {
  int nx = 0;
  bool has1 = false;
  for (int k = 0; k < n; ++k)
    for (int q = dep_rp[k]; q < dep_rp[k + 1]; ++q) {
      const int d = lower ? k - dep_ci[q] : dep_ci[q] - k;
      if (d <= 0) return 0;
      if (d == 1) { has1 = true; continue; }
      if (nx == 0) nx = d;
      else if (d != nx) return 0;
    }
  if (nx == 0) nx = has1 ? n : 0;
  if (nx < 2 || n % nx != 0) return 0;
  for (int k = 0; k < n; ++k)
    for (int q = dep_rp[k]; q < dep_rp[k + 1]; ++q) {
      const int d = lower ? k - dep_ci[q] : dep_ci[q] - k;
      if (d == 1 && (lower ? k % nx == 0 : k % nx == nx - 1)) return 0;  // crosses a grid row
    }
  return nx;
}

// (nx, ny) of a 3D grid: every dependency of row k is k -+ 1 within a grid
// line of nx cells, k -+ nx within a plane of nx * ny cells or k -+ nx * ny,
// all three offsets occur, and there are at least two planes; false otherwise
static bool grid3d_dims(int n, const std::vector<int>& dep_rp, const std::vector<int>& dep_ci, bool lower, int& gx,
                        int& gy) {
  int d1 = 0, d2 = 0, d3 = 0;  // the distinct offsets, ascending
  for (int k = 0; k < n; ++k)
    for (int q = dep_rp[k]; q < dep_rp[k + 1]; ++q) {
      const int d = lower ? k - dep_ci[q] : dep_ci[q] - k;
      if (d <= 0) return false;
      if (d == d1 || d == d2 || d == d3) continue;
      if (d3 != 0) return false;  // a fourth offset
      if (d1 == 0 || d < d1) { d3 = d2; d2 = d1; d1 = d; }
      else if (d2 == 0 || d < d2) { d3 = d2; d2 = d; }
      else d3 = d;
    }
  if (d1 != 1 || d2 < 2 || d3 <= d2 || d3 % d2 != 0 || n % d3 != 0 || n / d3 < 2) return false;
  const int nx = d2, nxy = d3;
  for (int k = 0; k < n; ++k)
    for (int q = dep_rp[k]; q < dep_rp[k + 1]; ++q) {
      const int d = lower ? k - dep_ci[q] : dep_ci[q] - k;
      if (d == 1 && (lower ? k % nx == 0 : k % nx == nx - 1)) return false;                 // crosses a grid line
      if (d == nx && (lower ? k % nxy < nx : k % nxy >= nxy - nx)) return false;           // crosses a plane
    }
  gx = nx;
  gy = nxy / nx;
  return true;
}

static int wave_cell_host(int64_t q, const WaveGrid& g) {
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

// Lay a factor out for the wavefront sweep: values from vals_dev (entries
// dep_src), reciprocal diagonal from dinv_dev (natural order) when given.
static void build_wave(WaveSweep& f, const WaveGrid& g, const std::vector<int>& dep_rp,
                       const std::vector<int>& dep_ci, const std::vector<int>& dep_src, bool lower,
                       const double* vals_dev, int64_t nvals, const double* dinv_dev, int n, hipStream_t s) {
  f.has_diag = dinv_dev != nullptr;
  if (g.nz > 0) {
    // quads (z, y, x neighbour, reciprocal diagonal) gathered from one buffer:
    // the factor's values, then the reciprocal diagonal, then a zero
    const int64_t T4 = 4 * g.total;
    const int64_t zero = nvals + n;
    const int nx = g.nx, nxy = g.nx * g.ny;
    std::vector<int> qidx(T4);
    parallel_ranges((int)g.total, [&](int p0, int p1, int) {
      for (int64_t p = p0; p < p1; ++p) {
        const int c = wave_cell_host(lower ? p : g.total - 1 - p, g);
        int iz = (int)zero, iy = (int)zero, ix = (int)zero, id = (int)zero;
        if (c >= 0) {
          const int cz = lower ? c - nxy : c + nxy, cy = lower ? c - nx : c + nx, cx = lower ? c - 1 : c + 1;
          for (int q = dep_rp[c]; q < dep_rp[c + 1]; ++q) {
            if (dep_ci[q] == cz) iz = dep_src[q];
            if (dep_ci[q] == cy) iy = dep_src[q];
            if (dep_ci[q] == cx) ix = dep_src[q];
          }
          if (f.has_diag) id = (int)(nvals + c);
        }
        qidx[4 * p] = iz;
        qidx[4 * p + 1] = iy;
        qidx[4 * p + 2] = ix;
        qidx[4 * p + 3] = id;
      }
    });
    DBuf<double> src;
    src.alloc(zero + 1);
    d2d(src.p, vals_dev, nvals, s);
    if (f.has_diag) d2d(src.p + nvals, dinv_dev, n, s);
    else launch_fill_f64_bits(src.p + nvals, 0ULL, n, s);
    launch_fill_f64_bits(src.p + zero, 0ULL, 1, s);
    DBuf<int> ix;
    ix.alloc(T4);
    h2d(ix.p, qidx.data(), T4, s);
    f.coef.alloc(T4);
    f.coef32.alloc(T4);
    launch_gather_f64(src.p, ix.p, f.coef.p, T4, s);
    launch_cast_f32(f.coef.p, f.coef32.p, T4, s);
    HIPCK(hipStreamSynchronize(s));
    return;
  }
  const int64_t T2 = 2 * g.total;
  std::vector<int> cidx(T2), didx(f.has_diag ? g.total : 0);
  parallel_ranges((int)g.total, [&](int p0, int p1, int) {
    for (int64_t p = p0; p < p1; ++p) {
      const int c = wave_cell_host(lower ? p : g.total - 1 - p, g);
      int below = (int)nvals, left = (int)nvals;  // index nvals: zero
      if (c >= 0) {
        const int cb = lower ? c - g.nx : c + g.nx, cl = lower ? c - 1 : c + 1;
        for (int q = dep_rp[c]; q < dep_rp[c + 1]; ++q) {
          if (dep_ci[q] == cb) below = dep_src[q];
          if (dep_ci[q] == cl) left = dep_src[q];
        }
      }
      cidx[2 * p] = below;
      cidx[2 * p + 1] = left;
      if (f.has_diag) didx[p] = c >= 0 ? c : n;
    }
  });
  DBuf<double> vz;
  vz.alloc(nvals + 1);
  d2d(vz.p, vals_dev, nvals, s);
  launch_fill_f64_bits(vz.p + nvals, 0ULL, 1, s);
  DBuf<int> ix;
  ix.alloc(T2);
  h2d(ix.p, cidx.data(), T2, s);
  f.coef.alloc(T2);
  f.coef32.alloc(T2);
  launch_gather_f64(vz.p, ix.p, f.coef.p, T2, s);
  launch_cast_f32(f.coef.p, f.coef32.p, T2, s);
  if (f.has_diag) {
    DBuf<double> dz;
    dz.alloc((size_t)n + 1);
    d2d(dz.p, dinv_dev, n, s);
    launch_fill_f64_bits(dz.p + n, 0ULL, 1, s);
    DBuf<int> dx;
    dx.alloc(g.total);
    h2d(dx.p, didx.data(), g.total, s);
    f.dinv.alloc(g.total);
    f.dinv32.alloc(g.total);
    launch_gather_f64(dz.p, dx.p, f.dinv.p, g.total, s);
    launch_cast_f32(f.dinv.p, f.dinv32.p, g.total, s);
    HIPCK(hipStreamSynchronize(s));
  }
  HIPCK(hipStreamSynchronize(s));
}

static void setup_impl(Solver& S, int64_t n64, int64_t nnz64, const int32_t* rowptr, const int32_t* col,
                       const double* val) {
  hipStream_t s = S.s;
  if (n64 <= 0 || n64 >= (1LL << 31) - 64 || nnz64 < n64 || nnz64 >= (1LL << 31))
    fail(GMG_ERR_INVALID_ARG, "setup: need 0 < n, n <= nnz < 2^31");
  if (!rowptr || !col || !val) fail(GMG_ERR_INVALID_ARG, "setup: null matrix pointer");
  const gmg_options& o = S.opt;
  if (!(o.cf >= 1.0) || o.max_passes < 0 || o.match_qbits < 0 || o.match_qbits > 52 || !(o.ilut_tau >= 0.0) ||
      o.coarse_mode < 0 || o.coarse_mode > 3 || o.coarse_sweeps < 0 || o.sweep_waves < 0 ||
      o.coarse_order < 0 || o.coarse_order > 1 || o.sweep_kernel < 0 || o.sweep_kernel > 3 ||
      o.sweep_wg_chunks < 0 || o.fine_order < 0 || o.fine_order > 2)
    fail(GMG_ERR_INVALID_ARG, "setup: option out of range");
  auto t0 = std::chrono::steady_clock::now();
  // GMG_LOG also prints the duration of each setup phase (it then waits for
  // the stream at every phase boundary, which normal runs never do)
  auto tp = t0;
  auto phase = [&](const char* what) {
    if (S.log_every <= 0) return;
    HIPCK(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[gmg] setup %-22s %9.2f ms\n", what, std::chrono::duration<double, std::milli>(now - tp).count());
    tp = now;
  };
  const int n = (int)n64;
  S.n = n;
  S.nnz = nnz64;
  HIPCK(hipHostMalloc(&S.hpin, sizeof(double) * 3 * kPinCol, hipHostMallocDefault));
  for (auto& e : S.colev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  S.abort_flag.alloc(1);
  launch_fill_u32(reinterpret_cast<unsigned*>(S.abort_flag.p), 0u, 1, s);
  // ---- validate and copy A
  {
    int64_t rp_end = 0;
    int first = 0;
    int rpn = 0;
    d2h(&first, rowptr, 1, s);
    d2h(&rpn, rowptr + n, 1, s);
    HIPCK(hipStreamSynchronize(s));
    rp_end = rpn;
    if (first != 0 || rp_end != nnz64) fail(GMG_ERR_INVALID_ARG, "setup: rowptr[0] != 0 or rowptr[n] != nnz");
  }
  DBuf<int> flags;
  flags.alloc(2);
  launch_fill_u32(reinterpret_cast<unsigned*>(flags.p), 0u, 2, s);
  launch_validate(n, rowptr, col, val, flags.p, s);
  int hflags[2] = {0, 0};
  d2h(hflags, flags.p, 2, s);
  HIPCK(hipStreamSynchronize(s));
  if (hflags[0]) fail(GMG_ERR_INVALID_ARG, "setup: columns must be in range, strictly ascending, diagonal stored");
  if (hflags[1]) fail(GMG_ERR_NONFINITE, "setup: non-finite matrix entry");
  S.A.n = S.A.m = n;
  S.A.nnz = nnz64;
  S.A.rp.alloc(n + 1);
  S.A.ci.alloc(nnz64);
  S.A.v.alloc(nnz64);
  S.A.v32.alloc(nnz64);
  d2d(S.A.rp.p, rowptr, n + 1, s);
  d2d(S.A.ci.p, col, nnz64, s);
  d2d(S.A.v.p, val, nnz64, s);
  launch_cast_f32(S.A.v.p, S.A.v32.p, nnz64, s);
  // ---- A^T (graph, adjoint)
  S.AT.n = S.AT.m = n;
  S.AT.nnz = nnz64;
  transpose_csr(n, n, nnz64, S.A.rp.p, S.A.ci.p, S.A.v.p, S.AT.rp, S.AT.ci, &S.AT.v, &S.at_src, s);
  phase("validate+transpose");
  // ---- aggregation
  {
    DBuf<int> grp, gci;
    DBuf<double> gw;
    build_graph(n, S.A.rp.p, S.A.ci.p, S.A.v.p, S.AT.rp.p, S.AT.ci.p, S.AT.v.p, grp, gci, gw, s);
    S.nc = aggregate(n, grp, gci, gw, o.cf, o.max_passes, o.match_qbits, o.hash_seed, S.agg, &S.passes,
                     &S.rounds, s);
  }
  phase("matching");
  build_members(n, S.nc, S.agg.p, S.aptr, S.amem, s);
  galerkin(n, S.nc, S.A.rp.p, S.A.ci.p, S.A.v.p, S.agg.p, S.aptr.p, S.amem.p, S.Ac, s);
  phase("galerkin");
  // ---- the coarse chain on a second host thread, while the fine level is
  // set up below: the nested-dissection numbering of the aggregates (A_c
  // rebuilt in that order), then the ILUT (or SPAI) of A_c on the host
  // threads.  Both threads queue work on the stream; the buffers each one
  // touches are disjoint (the coarse chain: agg, the members, A_c, the
  // dissection tree and the host factors).
  if (o.coarse_mode == 3 && S.nc > kDenseMaxCoarse)
    fail(GMG_ERR_INVALID_ARG, "coarse_mode 3 (dense inverse) needs n_coarse <= 8192");
  gmg_status ilut_st = GMG_OK;
  std::exception_ptr coarse_err;
  HCsr hAc;
  struct Joiner {  // joins on every path out of the setup, failures included
    std::thread t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } coarse_job;
  coarse_job.t = std::thread([&S, &hAc, &ilut_st, &coarse_err, n, s, tau = o.ilut_tau, mode = o.coarse_mode,
                              nd = o.coarse_order == 1] {
    try {
      PoolStream scope(s);
      if (nd && S.nc > 1) {
        // number the aggregates in nested-dissection order of A_c's graph,
        // then rebuild P^T and A_c (same sums, permuted rows and columns)
        const int nc = S.nc;
        // the graph of A_c + A_c^T without the diagonal, built on the device
        // (the same merge as the fine graph's; the weights are not needed)
        std::vector<int> cnt, gci;
        {
          DBuf<int> trp, tci, grp, gcd;
          DBuf<double> tv, gw;
          transpose_csr(nc, nc, S.Ac.nnz, S.Ac.rp.p, S.Ac.ci.p, S.Ac.v.p, trp, tci, &tv, nullptr, s);
          build_graph(nc, S.Ac.rp.p, S.Ac.ci.p, S.Ac.v.p, trp.p, tci.p, tv.p, grp, gcd, gw, s);
          cnt = to_host_int(grp.p, nc + 1, s);
          HIPCK(hipStreamSynchronize(s));
          gci = to_host_int(gcd.p, cnt[nc], s);
          HIPCK(hipStreamSynchronize(s));
        }
        std::vector<int> perm = nd_numbering(nc, cnt, gci, &S.nd_tree);
        std::vector<int> rank(nc);
        for (int k = 0; k < nc; ++k) rank[perm[k]] = k;
        DBuf<int> drank;
        drank.alloc(nc);
        h2d(drank.p, rank.data(), nc, s);
        relabel(n, S.agg.p, drank.p, s);
        HIPCK(hipStreamSynchronize(s));
        build_members(n, nc, S.agg.p, S.aptr, S.amem, s);
        galerkin(n, nc, S.A.rp.p, S.A.ci.p, S.A.v.p, S.agg.p, S.aptr.p, S.amem.p, S.Ac, s);
      }
      hAc.n = S.nc;
      hAc.rp = to_host_int(S.Ac.rp.p, S.nc + 1, s);
      hAc.ci = to_host_int(S.Ac.ci.p, S.Ac.nnz, s);
      hAc.v.resize(S.Ac.nnz);
      d2h_large(hAc.v.data(), S.Ac.v.p, S.Ac.nnz, s);
      HIPCK(hipStreamSynchronize(s));
      ilut_st = mode == 3   ? GMG_OK
                : mode == 2 ? host_spai(hAc, S.hMc)
                            : host_ilut(hAc, tau, S.hLc, S.hUc, &S.nd_tree);
    } catch (...) {
      coarse_err = std::current_exception();
    }
  });
  // ---- host copy of A's pattern for the analysis
  std::vector<int> hrp = to_host_int(S.A.rp.p, n + 1, s);
  std::vector<int> hci = to_host_int(S.A.ci.p, nnz64, s);
  HIPCK(hipStreamSynchronize(s));
  {
    // entries of A's largest 256-row tile: the SpMV's LDS capacity
    int64_t mt = 0;
    for (int r0 = 0; r0 < n; r0 += 256) mt = std::max<int64_t>(mt, hrp[std::min(n, r0 + 256)] - hrp[r0]);
    S.spmv_cap = spmv_cap(mt);
  }
  // ---- GMG-ND / multicolour: the smoother works on F = Q A Q^T, Q the
  // nested-dissection numbering of A's graph (the coarse numbering's rule) or
  // its colour classes; from here on hrp/hci hold F's pattern
  const int* frp_dev = S.A.rp.p;
  const int* fci_dev = S.A.ci.p;
  const double* fval_dev = S.A.v.p;
  DBuf<double> fval;
  if (o.fine_order >= 1) {
    std::vector<int> cnt(n + 1, 0);
    for (int i = 0; i < n; ++i)
      for (int p = hrp[i]; p < hrp[i + 1]; ++p)
        if (hci[p] != i) { cnt[i + 1]++; cnt[hci[p] + 1]++; }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int> gci(cnt[n]), fillp(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int p = hrp[i]; p < hrp[i + 1]; ++p)
        if (hci[p] != i) { gci[fillp[i]++] = hci[p]; gci[fillp[hci[p]]++] = i; }
    std::vector<int> perm = o.fine_order == 1 ? nd_numbering(n, cnt, gci, &S.fnd_tree) : color_numbering(n, cnt, gci);
    std::vector<int> rank(n), brp(n + 1, 0), bci(nnz64), bsrc(nnz64);
    for (int k = 0; k < n; ++k) rank[perm[k]] = k;
    for (int k = 0; k < n; ++k) brp[k + 1] = brp[k] + hrp[perm[k] + 1] - hrp[perm[k]];
    parallel_ranges(n, [&](int k0, int k1, int) {
      std::vector<std::pair<int, int>> row;
      for (int k = k0; k < k1; ++k) {
        const int i = perm[k];
        row.clear();
        for (int p = hrp[i]; p < hrp[i + 1]; ++p) row.emplace_back(rank[hci[p]], p);
        std::sort(row.begin(), row.end());
        for (size_t q = 0; q < row.size(); ++q) {
          bci[brp[k] + q] = row[q].first;
          bsrc[brp[k] + q] = row[q].second;
        }
      }
    });
    S.fperm.alloc(n);
    S.frp.alloc(n + 1);
    S.fci.alloc(nnz64);
    fval.alloc(nnz64);
    h2d(S.fperm.p, perm.data(), n, s);
    h2d(S.frp.p, brp.data(), n + 1, s);
    h2d(S.fci.p, bci.data(), nnz64, s);
    {
      DBuf<int> dsrc;
      dsrc.alloc(nnz64);
      h2d(dsrc.p, bsrc.data(), nnz64, s);
      launch_gather_f64(S.A.v.p, dsrc.p, fval.p, nnz64, s);
      HIPCK(hipStreamSynchronize(s));
    }
    hrp.swap(brp);
    hci.swap(bci);
    frp_dev = S.frp.p;
    fci_dev = S.fci.p;
    fval_dev = fval.p;
    S.fine_nd = true;
    phase(o.fine_order == 1 ? "fine nested dissection" : "fine colouring");
  }
  // diagonal positions and the dependency lists of the two forward fine
  // sweeps (strict lower / strict upper entries of each row): counts and
  // lists by row ranges on the host threads (the ILUT started above shares
  // them for these few milliseconds)
  std::vector<int> hdpos(n), l_rp(n + 1, 0), u_rp(n + 1, 0);
  parallel_ranges(n, [&](int i0, int i1, int) {
    for (int i = i0; i < i1; ++i) {
      int nl = 0, nu = 0;
      for (int p = hrp[i]; p < hrp[i + 1]; ++p) {
        if (hci[p] < i) ++nl;
        else if (hci[p] > i) ++nu;
        else hdpos[i] = p;
      }
      l_rp[i + 1] = nl;
      u_rp[i + 1] = nu;
    }
  });
  for (int i = 0; i < n; ++i) {
    l_rp[i + 1] += l_rp[i];
    u_rp[i + 1] += u_rp[i];
  }
  S.dpos.alloc(n);
  h2d(S.dpos.p, hdpos.data(), n, s);
  std::vector<int> l_ci(l_rp[n]), l_src(l_rp[n]), u_ci(u_rp[n]), u_src(u_rp[n]);
  parallel_ranges(n, [&](int i0, int i1, int) {
    for (int i = i0; i < i1; ++i) {
      int ql = l_rp[i], qu = u_rp[i];
      for (int p = hrp[i]; p < hrp[i + 1]; ++p) {
        const int c = hci[p];
        if (c < i) { l_ci[ql] = c; l_src[ql++] = p; }
        else if (c > i) { u_ci[qu] = c; u_src[qu++] = p; }
      }
    }
  });
  phase("fine dependency lists");
  // 2D-grid structure of both fine factors (their transposes then have it
  // too: the same offsets, mirrored): wavefront sweeps, and an ILU(0) in one
  // launch over the grid's anti-diagonals
  int grid_nx = 0, grid3_nx = 0, grid3_ny = 0;
  if ((o.sweep_kernel == 0 || o.sweep_kernel == 3) && !S.fine_nd) {
    const int nx = grid2d_nx(n, l_rp, l_ci, true);
    if (nx > 0 && grid2d_nx(n, u_rp, u_ci, false) == nx) grid_nx = nx;
    int lx = 0, ly = 0, ux = 0, uy = 0;
    if (grid_nx == 0 && grid3d_dims(n, l_rp, l_ci, true, lx, ly) && grid3d_dims(n, u_rp, u_ci, false, ux, uy) &&
        lx == ux && ly == uy) {
      grid3_nx = lx;
      grid3_ny = ly;
    }
  }
  // ---- ILU(0)
  S.ilu.alloc(nnz64);
  d2d(S.ilu.p, fval_dev, nnz64, s);
  {
    DBuf<int> bad;
    bad.alloc(1);
    launch_fill_u32(reinterpret_cast<unsigned*>(bad.p), 0u, 1, s);
    if (grid_nx > 0 && ilu0_grid_fits(grid_nx, n / grid_nx)) {
      launch_ilu0_grid(n, grid_nx, frp_dev, fci_dev, S.dpos.p, S.ilu.p, bad.p, s);
    } else {
      // one launch per level of L0
      std::vector<int> sched, lptr;
      int levels = 0;
      make_schedule(l_rp, l_ci, true, sched, lptr, &levels);
      DBuf<int> dsched;
      dsched.alloc(sched.size() > 0 ? sched.size() : 1);
      h2d(dsched.p, sched.data(), sched.size(), s);
      for (int l = 0; l < levels; ++l)
        launch_ilu0_level(dsched.p + lptr[l], lptr[l + 1] - lptr[l], frp_dev, fci_dev, S.dpos.p, S.ilu.p, bad.p, s);
      HIPCK(hipStreamSynchronize(s));
    }
    int hb = 0;
    d2h(&hb, bad.p, 1, s);
    HIPCK(hipStreamSynchronize(s));
    if (hb & 1) fail(GMG_ERR_ZERO_PIVOT, "ILU(0): zero pivot");
    if (hb & 2) fail(GMG_ERR_NONFINITE, "ILU(0): non-finite pivot");
  }
  phase("ILU(0)");
  S.u0dinv.alloc(n);
  hipLaunchKernelGGL(k_recip_diag, dim3((n + 255) / 256), dim3(256), 0, s, n, S.ilu.p, S.dpos.p, S.u0dinv.p);
  HIPCK(hipGetLastError());
  // wavefront form when both fine factors have 2D- or 3D-grid structure;
  // else the level-scheduled sweeps
  S.wave = false;
  if (grid_nx > 0) {
    const int nx = grid_nx;
    {
      WaveGrid& g = S.wg;
      g.nx = nx;
      g.ny = n / nx;
      g.W = (g.ny + 63) / 64;
      g.S = (nx + 63 + 15) / 16 * 16;  // whole pairs of chunks of the wavefront kernel
      g.total = (int64_t)g.W * g.S * 64;
      build_wave(S.wL0, g, l_rp, l_ci, l_src, true, S.ilu.p, nnz64, nullptr, n, s);
      build_wave(S.wU0, g, u_rp, u_ci, u_src, false, S.ilu.p, nnz64, S.u0dinv.p, n, s);
      S.wz.alloc(g.total); S.wy.alloc(g.total); S.wt.alloc(g.total);
      S.wz32.alloc(g.total); S.wy32.alloc(g.total); S.wt32.alloc(g.total);
      S.wave = true;
      // sizes and depths of the factors (profiling byte counts, info)
      S.L0.n = S.U0.n = n;
      S.L0.nnz = (int64_t)l_ci.size();
      S.U0.nnz = (int64_t)u_ci.size();
      S.U0.has_diag = true;
      S.L0.levels = S.U0.levels = g.nx + g.ny - 1;
      phase("wavefront layout");
    }
  } else if (grid3_nx > 0) {
    WaveGrid& g = S.wg;
    g.nx = grid3_nx;
    g.ny = grid3_ny;
    g.nz = n / (grid3_nx * grid3_ny);
    g.TY = (g.ny + 7) / 8;
    g.W = g.TY * ((g.nz + 7) / 8);
    g.S = (g.nx + 14 + 7) / 8 * 8;  // whole pairs of chunks of the 3D kernel
    g.total = (int64_t)g.W * g.S * 64;
    if (g.total < INT32_MAX / 4 && nnz64 + n < INT32_MAX) {
      build_wave(S.wL0, g, l_rp, l_ci, l_src, true, S.ilu.p, nnz64, nullptr, n, s);
      build_wave(S.wU0, g, u_rp, u_ci, u_src, false, S.ilu.p, nnz64, S.u0dinv.p, n, s);
      S.wz.alloc(g.total); S.wy.alloc(g.total); S.wt.alloc(g.total);
      S.wz32.alloc(g.total); S.wy32.alloc(g.total); S.wt32.alloc(g.total);
      S.wave = true;
      S.L0.n = S.U0.n = n;
      S.L0.nnz = (int64_t)l_ci.size();
      S.U0.nnz = (int64_t)u_ci.size();
      S.U0.has_diag = true;
      S.L0.levels = S.U0.levels = g.nx + g.ny + g.nz - 2;
      phase("wavefront layout (3D)");
    } else {
      g = WaveGrid();
    }
  }
  if (S.fine_nd && o.fine_order == 1 && o.sweep_kernel == 0) {
    // ILU(0) of F follows the dissection tree as the coarse ILUT does: the
    // tree solves apply it when every node fits
    std::vector<double> hilu(nnz64), hud(n);
    d2h(hilu.data(), S.ilu.p, nnz64, s);
    d2h(hud.data(), S.u0dinv.p, n, s);
    HIPCK(hipStreamSynchronize(s));
    if (build_tree(S.tL0, S.fnd_tree, n, l_rp, l_ci, &l_src, 0, hilu, true, nullptr, s) &&
        build_tree(S.tU0, S.fnd_tree, n, u_rp, u_ci, &u_src, 0, hilu, false, &hud, s)) {
      S.ftree = true;
      S.fext.alloc(n);
      S.fext32.alloc(n);
      S.L0.n = S.U0.n = n;
      S.L0.nnz = (int64_t)l_ci.size();
      S.U0.nnz = (int64_t)u_ci.size();
      S.U0.has_diag = true;
      S.L0.levels = S.U0.levels = S.tL0.heights;
      phase("fine tree solves");
    } else {
      S.tL0 = TreeSolve();
      S.tU0 = TreeSolve();
    }
  }
  if (!S.wave && !S.ftree) {
    // the two layouts are independent host work: U0's on a second thread
    std::exception_ptr u_err;
    std::thread ut([&] {
      try {
        PoolStream scope(s);
        build_sweep(S.U0, n, u_rp, u_ci, u_src, nullptr, S.ilu.p, false, true, nullptr, S.u0dinv.p, o.sweep_wg_chunks,
                    o.sweep_kernel == 2, s);
      } catch (...) {
        u_err = std::current_exception();
      }
    });
    try {
      build_sweep(S.L0, n, l_rp, l_ci, l_src, nullptr, S.ilu.p, true, false, nullptr, nullptr, o.sweep_wg_chunks,
                  o.sweep_kernel == 2, s);
    } catch (...) {
      ut.join();
      throw;
    }
    ut.join();
    if (u_err) std::rethrow_exception(u_err);
    phase("fine sweeps");
  }
  if (S.fine_nd) {
    S.fzp.alloc(n);
    S.ftp.alloc(n);
    S.fzp32.alloc(n);
    S.ftp32.alloc(n);
  }
  // ---- the coarse chain started above
  coarse_job.t.join();
  if (coarse_err) std::rethrow_exception(coarse_err);
  if (o.coarse_mode == 3) {
    const int nc = S.nc;
    S.cnp = (nc + 63) / 64 * 64;
    const size_t nn = (size_t)S.cnp * S.cnp;
    S.cinv.alloc(nn);
    S.cinv32.alloc(nn);
    S.cbad.alloc(1);
    HIPCK(hipMemsetAsync(S.cbad.p, 0, sizeof(int), s));
    launch_dense_inverse(nc, S.cnp, S.Ac.rp.p, S.Ac.ci.p, S.Ac.v.p, S.cinv.p, S.cbad.p, s);
    launch_cast_f32(S.cinv.p, S.cinv32.p, nn, s);
    int bad = 0;
    HIPCK(hipMemcpyAsync(&bad, S.cbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (bad) fail(GMG_ERR_ZERO_PIVOT, "dense coarse inverse: zero or non-finite pivot");
    phase("coarse chain: dissection, dense inverse");
  } else if (o.coarse_mode == 2) {
    const gmg_status st = ilut_st;
    if (st == GMG_ERR_ZERO_PIVOT) fail(st, "SPAI: a column's least-squares problem is rank deficient");
    if (st != GMG_OK) fail(st, "SPAI: non-finite entry");
    const HCsr& M = S.hMc;
    DCsr& D = S.dMc;
    D.n = D.m = S.nc;
    D.nnz = (int64_t)M.ci.size();
    D.rp.alloc(S.nc + 1);
    D.ci.alloc(D.nnz > 0 ? D.nnz : 1);
    D.v.alloc(D.nnz > 0 ? D.nnz : 1);
    D.v32.alloc(D.nnz > 0 ? D.nnz : 1);
    h2d(D.rp.p, M.rp.data(), S.nc + 1, s);
    h2d(D.ci.p, M.ci.data(), D.nnz, s);
    h2d(D.v.p, M.v.data(), D.nnz, s);
    launch_cast_f32(D.v.p, D.v32.p, D.nnz, s);
    HIPCK(hipStreamSynchronize(s));
    phase("coarse chain: dissection, SPAI (rest)");
  } else {
    {
      const gmg_status st = ilut_st;
      if (st == GMG_ERR_ZERO_PIVOT) fail(st, "ILUT: zero pivot");
      if (st == GMG_ERR_OOM) fail(st, "ILUT: factor exceeds int32 indexing");
      if (st != GMG_OK) fail(st, "ILUT: non-finite pivot");
    }
    phase("coarse chain: dissection, ILUT (rest)");
    {
      const int nc = S.nc;
      const HCsr &L = S.hLc, &U = S.hUc;
      std::vector<double> udinv(nc);
      for (int i = 0; i < nc; ++i) udinv[i] = 1.0 / U.v[U.rp[i]];
      // tree solves when the coarse unknowns are in nested-dissection order and
      // both factors follow the tree (U without its leading diagonal entries);
      // else the level-scheduled sweeps
      S.tree = false;
      bool tree_ok = false;
      if (o.sweep_kernel == 0 && o.coarse_order == 1 && !S.nd_tree.empty()) {
        // the two layouts at once: U~'s on a second host thread and its own
        // stream (its inputs are host data only), so that the host work and
        // the blocks' inversions of the two factors overlap.  That thread
        // allocates outside the solver's allocation scope (directly from the
        // runtime), so it never waits for a cached block of the first stream.
        hipStream_t s2 = nullptr;
        HIPCK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        bool ok_u = false;
        std::exception_ptr u_err;
        std::thread ut([&] {
          try {
            ok_u = build_tree(S.tUc, S.nd_tree, nc, U.rp, U.ci, nullptr, 1, U.v, false, &udinv, s2);
          } catch (...) {
            u_err = std::current_exception();
          }
        });
        bool ok_l = false;
        std::exception_ptr l_err;
        try {
          ok_l = build_tree(S.tLc, S.nd_tree, nc, L.rp, L.ci, nullptr, 0, L.v, true, nullptr, s);
        } catch (...) {
          l_err = std::current_exception();
        }
        ut.join();
        (void)hipStreamSynchronize(s2);
        (void)hipStreamDestroy(s2);
        if (l_err) std::rethrow_exception(l_err);
        if (u_err) std::rethrow_exception(u_err);
        tree_ok = ok_l && ok_u;
      }
      if (tree_ok) {
        S.tree = true;
        S.text.alloc(nc);
        S.text32.alloc(nc);
        // sizes and depths (profiling byte counts, info)
        S.Lc.n = S.Uc.n = nc;
        S.Lc.nnz = (int64_t)L.ci.size();
        S.Uc.nnz = (int64_t)U.ci.size() - nc;
        S.Uc.has_diag = true;
        S.Lc.levels = S.Uc.levels = S.tLc.heights;
        phase("coarse tree solves");
      } else {
        S.tLc = TreeSolve();
        S.tUc = TreeSolve();
        std::vector<int> lsrc(L.ci.size()), us_rp(nc + 1, 0), us_ci, us_src;
        for (size_t q = 0; q < L.ci.size(); ++q) lsrc[q] = (int)q;
        for (int i = 0; i < nc; ++i) {
          for (int q = U.rp[i] + 1; q < U.rp[i + 1]; ++q) { us_ci.push_back(U.ci[q]); us_src.push_back(q); }
          us_rp[i + 1] = (int)us_ci.size();
        }
        build_sweep(S.Lc, nc, L.rp, L.ci, lsrc, &L.v, nullptr, true, false, nullptr, nullptr, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
        build_sweep(S.Uc, nc, us_rp, us_ci, us_src, &U.v, nullptr, false, true, &udinv, nullptr, o.sweep_wg_chunks, o.sweep_kernel == 2, s);
        phase("coarse sweeps");
      }
      if (o.coarse_mode == 1) {
        auto up = [&](DCsr& D, const HCsr& H) {
          D.n = D.m = nc;
          D.nnz = (int64_t)H.ci.size();
          D.rp.alloc(nc + 1);
          D.ci.alloc(D.nnz > 0 ? D.nnz : 1);
          D.v.alloc(D.nnz > 0 ? D.nnz : 1);
          h2d(D.rp.p, H.rp.data(), nc + 1, s);
          h2d(D.ci.p, H.ci.data(), D.nnz, s);
          h2d(D.v.p, H.v.data(), D.nnz, s);
        };
        up(S.dLc, L);
        up(S.dUc, U);
        S.ucdinv.alloc(nc);
        h2d(S.ucdinv.p, udinv.data(), nc, s);
        S.jzero.alloc(nc);
        S.jtmp.alloc(nc);
        HIPCK(hipMemsetAsync(S.jzero.p, 0, sizeof(double) * nc, s));
        HIPCK(hipStreamSynchronize(s));
      }
    }
  }
  // ---- work vectors
  S.y.alloc(n); S.t.alloc(n); S.r.alloc(n);
  S.rc.alloc(S.nc); S.yc.alloc(S.nc); S.ec.alloc(S.nc);
  S.y32.alloc(n); S.t32.alloc(n); S.r32.alloc(n);
  S.rc32.alloc(S.nc); S.yc32.alloc(S.nc); S.ec32.alloc(S.nc);
  S.abc.alloc(S.nc); S.auc.alloc(S.nc); S.aec.alloc(S.nc);
  S.as.alloc(n); S.aw.alloc(n); S.at.alloc(n);
  // staging of the single-CU sweeps, with the dummy entry at index n
  S.cu_rhs.alloc(std::max(n, S.nc) + 1); S.cu_out.alloc(std::max(n, S.nc) + 1);
  S.cu_rhs32.alloc(std::max(n, S.nc) + 1); S.cu_out32.alloc(std::max(n, S.nc) + 1);
  launch_fill_f64_bits(S.cu_rhs.p, 0ULL, std::max(n, S.nc) + 1, s);
  launch_fill_f32_bits(S.cu_rhs32.p, 0u, std::max(n, S.nc) + 1, s);
  red_init(S.rw, s);
  reset_cycle_buffers(S);
  HIPCK(hipStreamSynchronize(s));
  phase("work vectors");
  auto t1 = std::chrono::steady_clock::now();
  gmg_info& I = S.info;
  I.passes = S.passes;
  I.rounds = S.rounds;
  I.levels_L0 = S.L0.levels;
  I.levels_U0 = S.U0.levels;
  I.levels_Lc = S.Lc.levels;
  I.levels_Uc = S.Uc.levels;
  I.n = n;
  I.nnz = nnz64;
  I.n_coarse = S.nc;
  I.nnz_coarse = S.Ac.nnz;
  I.nnz_lc = (int64_t)S.hLc.ci.size();
  I.nnz_uc = (int64_t)S.hUc.ci.size();
  I.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace gmg

using gmg::Error;
using gmg::Solver;

struct gmg_solver {
  Solver S;
};

template <class F>
static gmg_status guarded(F&& f) {
  try {
    gmg::g_last_error.clear();
    return f();
  } catch (const Error& e) {
    gmg::g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    gmg::g_last_error = "host allocation failed";
    return GMG_ERR_OOM;
  } catch (const std::exception& e) {
    gmg::g_last_error = e.what();
    return GMG_ERR_HIP;
  }
}

#define REQUIRE_HANDLE(h)                                           \
  do {                                                              \
    if (!(h)) gmg::fail(GMG_ERR_NOT_SETUP, "null solver handle");   \
  } while (0)

extern "C" {

void gmg_default_options(gmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->cf = 4.0;
  o->max_passes = 8;
  o->match_qbits = 4;
  o->hash_seed = 0x9E3779B97F4A7C15ULL;
  o->ilut_tau = 1e-4;
  o->coarse_mode = 0;
  o->coarse_sweeps = 3;
  o->restart = 30;
  o->maxit = 600;
  o->precond_fp32 = 0;
  o->x0_given = 0;
  o->sweep_waves = 0;
  o->coarse_order = 1;
  o->sweep_kernel = 0;
  o->sweep_wg_chunks = 8;
  o->fine_order = 0;
}

gmg_status gmg_setup(gmg_handle* h, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                     const double* val, const gmg_options* opts, void* stream) {
  return guarded([&]() -> gmg_status {
    if (!h) gmg::fail(GMG_ERR_INVALID_ARG, "setup: null handle pointer");
    *h = nullptr;
    gmg::PoolStream pool_scope((hipStream_t)stream);
    std::unique_ptr<gmg_solver> sv(new gmg_solver());
    sv->S.s = (hipStream_t)stream;
    if (const char* e = std::getenv("GMG_LOG")) sv->S.log_every = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("GMG_COLUMN_LOOP")) sv->S.force_column_loop = std::atoi(e) != 0;
    if (opts) sv->S.opt = *opts;
    else gmg_default_options(&sv->S.opt);
    gmg::setup_impl(sv->S, n, nnz, rowptr, col, val);
    *h = sv.release();
    return GMG_OK;
  });
}

gmg_status gmg_solve(gmg_handle h, const double* b, double* x, int nrhs, double tol, const gmg_options* opts,
                     gmg_info* info) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    return gmg::solve_impl(h->S, false, b, x, nrhs, tol, opts, info);
  });
}

gmg_status gmg_solve_adjoint(gmg_handle h, const double* g, double* lambda, int nrhs, double tol,
                             const gmg_options* opts, gmg_info* info) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    return gmg::solve_impl(h->S, true, g, lambda, nrhs, tol, opts, info);
  });
}

gmg_status gmg_apply_precond(gmg_handle h, const double* z, double* q, int precision, int adjoint) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!z || !q) gmg::fail(GMG_ERR_INVALID_ARG, "apply: null vector");
    Solver& S = h->S;
    gmg::reset_cycle_buffers(S);
    if (adjoint) {
      if (precision != 0) gmg::fail(GMG_ERR_INVALID_ARG, "the adjoint apply runs in FP64 (precision 0)");
      gmg::vcycle_adjoint(S, z, q);
    } else if (precision == 1) {
      gmg::vcycle<float>(S, z, q);
    } else {
      gmg::vcycle<double>(S, z, q);
    }
    HIPCK(hipStreamSynchronize(S.s));
    gmg::check_abort(S);
    return GMG_OK;
  });
}

gmg_status gmg_spmv(gmg_handle h, int transposed, const double* x, double* y) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!x || !y) gmg::fail(GMG_ERR_INVALID_ARG, "spmv: null vector");
    gmg::apply_op(h->S, transposed != 0, x, y);
    HIPCK(hipStreamSynchronize(h->S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_info(gmg_handle h, gmg_info* info) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!info) gmg::fail(GMG_ERR_INVALID_ARG, "null info");
    *info = h->S.info;
    return GMG_OK;
  });
}

gmg_status gmg_get_history(gmg_handle h, int cap, double* hist, int* count) {
  return guarded([&]() -> gmg_status {
    if (!h || cap < 0 || !count || (cap > 0 && !hist)) gmg::fail(GMG_ERR_INVALID_ARG, "get_history: bad arguments");
    const auto& v = h->S.hist;
    *count = (int)v.size();
    std::copy(v.begin(), v.begin() + std::min<size_t>(v.size(), (size_t)cap), hist);
    return GMG_OK;
  });
}

gmg_status gmg_cond_estimate(gmg_handle h, double* est_coarse, double* est_ilut) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!est_coarse || !est_ilut) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    gmg::Solver& S = h->S;
    if (S.opt.coarse_mode >= 2) gmg::fail(GMG_ERR_INVALID_ARG, "no ILUT factors under coarse_mode 2 or 3");
    const int nc = S.nc;
    auto ratio = [](const std::vector<double>& d) {
      double mx = 0.0, mn = std::numeric_limits<double>::infinity();
      for (double v : d) { mx = std::max(mx, std::fabs(v)); mn = std::min(mn, std::fabs(v)); }
      return mn > 0.0 ? mx / mn : std::numeric_limits<double>::infinity();
    };
    // diagonal of A_c
    std::vector<int> rp = gmg::to_host_int(S.Ac.rp.p, nc + 1, S.s);
    std::vector<int> ci = gmg::to_host_int(S.Ac.ci.p, S.Ac.nnz, S.s);
    std::vector<double> v(S.Ac.nnz), dac(nc, 0.0);
    gmg::d2h(v.data(), S.Ac.v.p, S.Ac.nnz, S.s);
    HIPCK(hipStreamSynchronize(S.s));
    for (int i = 0; i < nc; ++i)
      for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) dac[i] = v[p];
    // diagonal of L~U~: u_ii + sum_{j<i} l_ij u_ji (U~'s rows: diagonal, then
    // ascending columns)
    const gmg::HCsr &L = S.hLc, &U = S.hUc;
    std::vector<double> dlu(nc, 0.0);
    for (int i = 0; i < nc; ++i) {
      double sum = U.v[U.rp[i]];
      for (int q = L.rp[i]; q < L.rp[i + 1]; ++q) {
        const int j = L.ci[q];
        const int* b = U.ci.data() + U.rp[j] + 1;
        const int* e = U.ci.data() + U.rp[j + 1];
        const int* f = std::lower_bound(b, e, i);
        if (f != e && *f == i) sum += L.v[q] * U.v[f - U.ci.data()];
      }
      dlu[i] = sum;
    }
    *est_coarse = ratio(dac);
    *est_ilut = ratio(dlu);
    return GMG_OK;
  });
}

gmg_status gmg_get_aggregates(gmg_handle h, int32_t* agg) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!agg) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    gmg::d2d(agg, h->S.agg.p, h->S.n, h->S.s);
    HIPCK(hipStreamSynchronize(h->S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_coarse(gmg_handle h, int32_t* rowptr, int32_t* col, double* val) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!rowptr || !col || !val) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    Solver& S = h->S;
    gmg::d2d(rowptr, S.Ac.rp.p, S.nc + 1, S.s);
    gmg::d2d(col, S.Ac.ci.p, S.Ac.nnz, S.s);
    gmg::d2d(val, S.Ac.v.p, S.Ac.nnz, S.s);
    HIPCK(hipStreamSynchronize(S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_ilu0(gmg_handle h, double* val) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!val) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    gmg::d2d(val, h->S.ilu.p, h->S.nnz, h->S.s);
    HIPCK(hipStreamSynchronize(h->S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_fine_perm(gmg_handle h, int32_t* perm) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!perm) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    gmg::Solver& S = h->S;
    if (S.fine_nd) {
      gmg::d2d(perm, S.fperm.p, S.n, S.s);
    } else {
      std::vector<int> id(S.n);
      for (int k = 0; k < S.n; ++k) id[k] = k;
      gmg::h2d(perm, id.data(), S.n, S.s);
    }
    HIPCK(hipStreamSynchronize(S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_spai(gmg_handle h, int32_t* rowptr, int32_t* col, double* val) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    gmg::Solver& S = h->S;
    if (S.opt.coarse_mode != 2) gmg::fail(GMG_ERR_INVALID_ARG, "no sparse approximate inverse (coarse_mode != 2)");
    if (!rowptr || !col || !val) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    gmg::d2d(rowptr, S.dMc.rp.p, S.nc + 1, S.s);
    gmg::d2d(col, S.dMc.ci.p, S.dMc.nnz, S.s);
    gmg::d2d(val, S.dMc.v.p, S.dMc.nnz, S.s);
    HIPCK(hipStreamSynchronize(S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_coarse_inverse(gmg_handle h, double* inv) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    gmg::Solver& S = h->S;
    if (S.opt.coarse_mode != 3) gmg::fail(GMG_ERR_INVALID_ARG, "no dense coarse inverse (coarse_mode != 3)");
    if (!inv) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    if (S.nc > 0)
      HIPCK(hipMemcpy2DAsync(inv, sizeof(double) * S.nc, S.cinv.p, sizeof(double) * S.cnp, sizeof(double) * S.nc,
                             S.nc, hipMemcpyDeviceToDevice, S.s));
    HIPCK(hipStreamSynchronize(S.s));
    return GMG_OK;
  });
}

gmg_status gmg_get_ilut(gmg_handle h, int32_t* lrp, int32_t* lci, double* lv, int32_t* urp, int32_t* uci,
                        double* uv) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    if (!lrp || !lci || !lv || !urp || !uci || !uv) gmg::fail(GMG_ERR_INVALID_ARG, "null output");
    Solver& S = h->S;
    gmg::h2d(lrp, S.hLc.rp.data(), S.hLc.rp.size(), S.s);
    gmg::h2d(lci, S.hLc.ci.data(), S.hLc.ci.size(), S.s);
    gmg::h2d(lv, S.hLc.v.data(), S.hLc.v.size(), S.s);
    gmg::h2d(urp, S.hUc.rp.data(), S.hUc.rp.size(), S.s);
    gmg::h2d(uci, S.hUc.ci.data(), S.hUc.ci.size(), S.s);
    gmg::h2d(uv, S.hUc.v.data(), S.hUc.v.size(), S.s);
    HIPCK(hipStreamSynchronize(S.s));
    return GMG_OK;
  });
}

gmg_status gmg_set_stream(gmg_handle h, void* stream) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    HIPCK(hipStreamSynchronize(h->S.s));
    gmg::pool_idle(h->S.s);
    h->S.s = (hipStream_t)stream;
    return GMG_OK;
  });
}

gmg_status gmg_profile_enable(gmg_handle h, int enable) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    Solver& S = h->S;
    gmg::prof_flush(S);
    for (int c = 0; c < gmg::PC_COUNT; ++c) { S.pc_launch[c] = 0; S.pc_ms[c] = 0; S.pc_bytes[c] = 0; }
    if (enable < 0) gmg::fail(GMG_ERR_INVALID_ARG, "profile: negative class mask");
    S.prof = enable != 0;
    S.prof_mask = enable == 1 ? ~0u : (unsigned)enable >> 1;
    return GMG_OK;
  });
}

gmg_status gmg_profile_read(gmg_handle h, int cap, int* count, int64_t* launches, double* ms, double* bytes) {
  return guarded([&]() -> gmg_status {
    REQUIRE_HANDLE(h);
    gmg::PoolStream pool_scope(h->S.s);
    Solver& S = h->S;
    gmg::prof_flush(S);
    if (count) *count = gmg::PC_COUNT;
    for (int c = 0; c < gmg::PC_COUNT && c < cap; ++c) {
      if (launches) launches[c] = S.pc_launch[c];
      if (ms) ms[c] = S.pc_ms[c];
      if (bytes) bytes[c] = S.pc_bytes[c];
    }
    return GMG_OK;
  });
}

const char* gmg_profile_name(int cls) {
  if (cls < 0 || cls >= gmg::PC_COUNT) return "";
  return gmg::kProfNames[cls];
}

void gmg_destroy(gmg_handle h) {
  if (!h) return;
  const hipStream_t s = h->S.s;
  (void)hipStreamSynchronize(s);
  {
    // everything queued on s has finished: the solver's memory goes back to
    // the cache, free for any stream
    gmg::PoolStream pool_scope(s);
    delete h;
  }
  gmg::pool_idle(s);
}

const char* gmg_last_error(void) { return gmg::g_last_error.c_str(); }

}  // extern "C"
