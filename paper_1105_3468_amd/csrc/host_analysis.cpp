// Host-side analysis steps of the setup: dependency-level schedules of the
// triangular factors, and the row-wise ILUT factorisation of the coarse matrix.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <condition_variable>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

#include "gmg_internal.h"

#pragma clang fp contract(off)

namespace gmg {

// level[r] = 1 + max level of its dependencies (0 without any); rows are
// listed level by level (ascending row index inside a level), every level
// padded with -1 to a multiple of 64 so one wave never spans two levels.
void make_schedule(const std::vector<int>& dep_rp, const std::vector<int>& dep_ci, bool lower,
                   std::vector<int>& sched, std::vector<int>& level_ptr, int* levels_out) {
  const int n = (int)dep_rp.size() - 1;
  std::vector<int> lev(n > 0 ? n : 1, 0);
  int nlev = 0;
  auto visit = [&](int r) {
    int l = 0;
    for (int q = dep_rp[r]; q < dep_rp[r + 1]; ++q) l = std::max(l, lev[dep_ci[q]] + 1);
    lev[r] = l;
    nlev = std::max(nlev, l + 1);
  };
  if (lower)
    for (int r = 0; r < n; ++r) visit(r);
  else
    for (int r = n - 1; r >= 0; --r) visit(r);
  if (n == 0) nlev = 0;
  std::vector<int> cnt(nlev + 1, 0);
  for (int r = 0; r < n; ++r) cnt[lev[r] + 1]++;
  std::vector<int> start(nlev + 1, 0);  // unpadded starts
  for (int l = 0; l < nlev; ++l) start[l + 1] = start[l] + cnt[l + 1];
  level_ptr.assign(nlev + 1, 0);
  for (int l = 0; l < nlev; ++l) {
    const int sz = cnt[l + 1];
    level_ptr[l + 1] = level_ptr[l] + ((sz + 63) / 64) * 64;
  }
  sched.assign(level_ptr[nlev], -1);
  std::vector<int> fill(level_ptr.begin(), level_ptr.end());
  for (int r = 0; r < n; ++r) sched[fill[lev[r]]++] = r;
  *levels_out = nlev;
}

// Row-wise ILUT(tau) without pivoting and without a fill limit.  For row i the
// drop threshold is tau * ||a_i||_2.  Candidates k < i are eliminated in
// ascending order (a min-priority queue tracks fill); a candidate is dropped
// when its value before the division by the pivot is below the threshold,
// otherwise it becomes the multiplier l_ik = w_k / u_kk and row k of U is
// subtracted.  U entries j > i below the threshold are dropped; the diagonal
// is always kept and stored first in its row.
//
// Row i reads only A's row i and the finished U rows of the k it eliminates.
// Under a nested-dissection numbering those rows lie in i's own tree node
// (earlier rows) or in its descendants, fill included: eliminating k adds
// columns of U's row k, which lie in k's node or its ancestors, all on the
// path through i's node.  So the nodes of the tree are factored as tasks, a
// node once all of its children are done, on a pool of threads.  Every row
// performs the same operations in the same order as in a row-by-row pass, so
// the factors are bit-identical to the sequential ones.
namespace {

struct IlutNodeRows {  // the factor rows [lo, hi) of one tree node
  int lo = 0;
  std::vector<int> lrp{0}, lci, urp{0}, uci;
  std::vector<double> lv, uv;
};

struct IlutWork {
  std::vector<double> w;
  std::vector<signed char> state;  // 0 absent, 1 present, 2 dropped
  std::vector<int> touched;        // every column set in this row (for the reset)
  std::vector<int> ucols;          // columns above the diagonal
  std::vector<int> kept;           // L columns, ascending (the eliminated, undropped candidates)
  std::vector<uint64_t> bits;      // pending candidates k < i (a set of column indices)
  int pos = 0;                     // no pending candidate below this column
  explicit IlutWork(int n)
      : w(n > 0 ? n : 1, 0.0), state(n > 0 ? n : 1, 0), bits((size_t)(n > 0 ? n : 1) / 64 + 1, 0) {
    touched.reserve(256);
    ucols.reserve(256);
    kept.reserve(256);
  }
  void add_pending(int j) { bits[(size_t)j >> 6] |= 1ull << (j & 63); }
  // the smallest pending candidate, or i when there is none (candidates are
  // all below i; an elimination only adds candidates above the one taken, so
  // the scan only moves forward)
  int next_pending(int i) {
    size_t wd = (size_t)pos >> 6;
    uint64_t m = bits[wd] & (~0ull << (pos & 63));
    const size_t last = (size_t)(i - 1) >> 6;
    while (m == 0) {
      if (i <= 0 || wd >= last) return i;
      m = bits[++wd];
    }
    const int k = (int)(wd * 64) + __builtin_ctzll(m);
    return k < i ? k : i;
  }
};

// A row's working state after the eliminations of the rows below its node.
struct IlutRowState {
  double thr = 0.0;
  std::vector<int> col, kept;
  std::vector<double> val;
  std::vector<signed char> st;
};

// Row i's start: A's row i in the work vector, its drop threshold, the
// candidates k < i pending.
double ilut_row_begin(const HCsr& A, double tau, int i, IlutWork& W) {
  double ss = 0.0;
  W.touched.clear();
  W.ucols.clear();
  W.kept.clear();
  W.pos = i;
  for (int p = A.rp[i]; p < A.rp[i + 1]; ++p) {
    const int j = A.ci[p];
    ss = ss + A.v[p] * A.v[p];
    W.w[j] = A.v[p];
    W.state[j] = 1;
    W.touched.push_back(j);
    if (j < i) {
      W.add_pending(j);
      W.pos = std::min(W.pos, j);
    } else if (j > i) {
      W.ucols.push_back(j);
    }
  }
  if (W.state[i] == 0) { W.state[i] = 1; W.w[i] = 0.0; W.touched.push_back(i); }
  return tau * std::sqrt(ss);
}

// Eliminations of the pending candidates k < until, in ascending order.
void ilut_row_eliminate(int i, double thr, int until, const std::vector<int>& node_of,
                        const std::vector<IlutNodeRows>& rows, IlutWork& W) {
  for (;;) {
    const int k = W.next_pending(i);
    if (k >= until) break;
    W.bits[(size_t)k >> 6] &= ~(1ull << (k & 63));
    W.pos = k + 1;
    if (std::fabs(W.w[k]) < thr) { W.w[k] = 0.0; W.state[k] = 2; continue; }
    const IlutNodeRows& K = rows[node_of[k]];
    const int uk = K.urp[k - K.lo], ue = K.urp[k - K.lo + 1];
    const int* uci = K.uci.data();
    const double* uv = K.uv.data();
    const double lik = W.w[k] / uv[uk];
    W.w[k] = lik;
    W.kept.push_back(k);
    for (int r = uk + 1; r < ue; ++r) {
      const int j = uci[r];
      if (W.state[j] == 0) {
        W.state[j] = 1;
        W.w[j] = 0.0;
        W.touched.push_back(j);
        if (j < i) W.add_pending(j);
        else if (j > i) W.ucols.push_back(j);
      }
      W.w[j] = W.w[j] - lik * uv[r];
    }
  }
}

// Save a row's state (its pending candidates are exactly its present
// columns in [until, i)) and clear the work vector; restore it for the rest.
void ilut_row_save(int i, int until, double thr, IlutWork& W, IlutRowState& R) {
  R.thr = thr;
  R.col.assign(W.touched.begin(), W.touched.end());
  R.kept.assign(W.kept.begin(), W.kept.end());
  R.val.resize(R.col.size());
  R.st.resize(R.col.size());
  for (size_t q = 0; q < R.col.size(); ++q) {
    const int j = R.col[q];
    R.val[q] = W.w[j];
    R.st[q] = W.state[j];
    if (W.state[j] == 1 && j >= until && j < i) W.bits[(size_t)j >> 6] &= ~(1ull << (j & 63));
    W.w[j] = 0.0;
    W.state[j] = 0;
  }
}
double ilut_row_restore(int i, int from, const IlutRowState& R, IlutWork& W) {
  W.touched.assign(R.col.begin(), R.col.end());
  W.kept.assign(R.kept.begin(), R.kept.end());
  W.ucols.clear();
  W.pos = i;
  for (size_t q = 0; q < R.col.size(); ++q) {
    const int j = R.col[q];
    W.w[j] = R.val[q];
    W.state[j] = R.st[q];
    if (R.st[q] == 1 && j >= from && j < i) {
      W.add_pending(j);
      W.pos = std::min(W.pos, j);
    } else if (j > i) {
      W.ucols.push_back(j);
    }
  }
  return R.thr;
}

// Row i's end: drops, the split into L (the kept candidates, ascending) and U
// (diagonal first, then ascending columns), the work vector cleared.  Returns
// false (status in *st) on a zero or non-finite pivot.
bool ilut_row_finish(int i, double thr, IlutWork& W, IlutNodeRows& R, gmg_status* st) {
  for (int j : W.kept) {
    R.lci.push_back(j);
    R.lv.push_back(W.w[j]);
  }
  const double d = W.w[i];
  R.uci.push_back(i);
  R.uv.push_back(d);
  std::sort(W.ucols.begin(), W.ucols.end());
  for (int j : W.ucols)
    if (!(std::fabs(W.w[j]) < thr)) { R.uci.push_back(j); R.uv.push_back(W.w[j]); }
  for (int j : W.touched) {
    W.state[j] = 0;
    W.w[j] = 0.0;
  }
  R.lrp.push_back((int)R.lci.size());
  R.urp.push_back((int)R.uci.size());
  if (d == 0.0) { *st = GMG_ERR_ZERO_PIVOT; return false; }
  if (!std::isfinite(d)) { *st = GMG_ERR_NONFINITE; return false; }
  return true;
}

}  // namespace

int host_threads() {
  static const int t = [] {
    const char* e = std::getenv("GMG_THREADS");
    if (!e || !*e) e = std::getenv("OMP_NUM_THREADS");
    int v = e ? std::atoi(e) : 0;
    if (v <= 0) v = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(v, 64));
  }();
  return t;
}

gmg_status host_ilut(const HCsr& A, double tau, HCsr& L, HCsr& U, const std::vector<NdNode>* tree) {
  const int n = A.n;
  L.n = U.n = n;
  // tasks: the tree's nonempty nodes, or one task over all rows
  std::vector<int> lo, hi, parent;
  std::vector<int> node_of(n > 0 ? n : 1, -1);
  bool use_tree = tree && !tree->empty() && host_threads() > 1;
  if (use_tree) {
    const int nn = (int)tree->size();
    std::vector<int> task_of(nn, -1);
    for (int k = 0; k < nn; ++k) {
      const NdNode& d = (*tree)[k];
      if (d.lo < 0 || d.hi > n || d.lo > d.hi) { use_tree = false; break; }
      task_of[k] = (int)lo.size();
      lo.push_back(d.lo);
      hi.push_back(d.hi);
      for (int r = d.lo; r < d.hi; ++r) {
        if (node_of[r] >= 0) use_tree = false;
        node_of[r] = task_of[k];
      }
    }
    for (int r = 0; r < n && use_tree; ++r)
      if (node_of[r] < 0) use_tree = false;
    if (use_tree) {
      // a node's parent is the task of its tree parent (empty nodes included:
      // they are trivial tasks and keep the dependency chain intact)
      parent.assign(lo.size(), -1);
      for (int k = 0; k < nn; ++k) parent[task_of[k]] = (*tree)[k].parent >= 0 ? task_of[(*tree)[k].parent] : -1;
    }
  }
  if (!use_tree) {
    lo.assign(1, 0);
    hi.assign(1, n);
    parent.assign(1, -1);
    std::fill(node_of.begin(), node_of.end(), 0);
  }
  const int nt = (int)lo.size();
  std::vector<IlutNodeRows> rows(nt);
  for (int k = 0; k < nt; ++k) {
    rows[k].lo = lo[k];
    rows[k].lrp.reserve(hi[k] - lo[k] + 1);
    rows[k].urp.reserve(hi[k] - lo[k] + 1);
  }
  std::vector<int> fail_row(nt, -1);
  std::vector<gmg_status> fail_st(nt, GMG_OK);
  // whole rows of a node, stopping at the first failing one
  auto full_rows = [&](int k, IlutWork& W) {
    for (int i = lo[k]; i < hi[k]; ++i) {
      const double thr = ilut_row_begin(A, tau, i, W);
      ilut_row_eliminate(i, thr, i, node_of, rows, W);
      if (!ilut_row_finish(i, thr, W, rows[k], &fail_st[k])) {
        fail_row[k] = i;
        return;
      }
    }
  };
  if (nt == 1) {
    IlutWork W(n);
    full_rows(0, W);
  } else {
    // Jobs: a node's rows in one go; or, for a large node with descendants,
    // phase 1 (the eliminations of rows below the node, whose U rows are all
    // final once the children are done: independent across the node's rows,
    // so cut into chunks) and phase 2 (the node's own eliminations, row by
    // row, from the saved states).  Each row runs the same operations in the
    // same order either way.
    constexpr int kSplitRows = 48, kChunkRows = 16;
    struct Job { int kind, node, r0, r1; };  // kind 0: whole node, 1: phase 1 of rows [r0, r1), 2: phase 2
    std::vector<Job> jobs;
    std::vector<int> first_job(nt), n_first(nt), phase2(nt, -1), p1_left(nt, 0);
    std::vector<std::vector<IlutRowState>> saved(nt);
    std::vector<int> nkids(nt, 0);
    for (int k = 0; k < nt; ++k)
      if (parent[k] >= 0) nkids[parent[k]]++;
    for (int k = 0; k < nt; ++k) {
      first_job[k] = (int)jobs.size();
      const int nr = hi[k] - lo[k];
      if (nr >= kSplitRows && nkids[k] > 0) {
        for (int r = lo[k]; r < hi[k]; r += kChunkRows) jobs.push_back({1, k, r, std::min(hi[k], r + kChunkRows)});
        n_first[k] = (int)jobs.size() - first_job[k];
        p1_left[k] = n_first[k];
        phase2[k] = (int)jobs.size();
        jobs.push_back({2, k, lo[k], hi[k]});
        saved[k].resize(nr);
      } else {
        jobs.push_back({0, k, lo[k], hi[k]});
        n_first[k] = 1;
      }
    }
    std::vector<int> waiting(nkids);
    std::vector<char> poisoned(nt, 0);
    // ready jobs by the estimated length of their node's path to the root (a
    // node costs about rows^1.5 here), longest first; a parent precedes its
    // children in the task order
    std::vector<double> prio(nt, 0.0);
    for (int k = 0; k < nt; ++k) {
      const double nr = (double)(hi[k] - lo[k]);
      prio[k] = nr * std::sqrt(nr) + (parent[k] >= 0 && parent[k] < k ? prio[parent[k]] : 0.0);
    }
    std::priority_queue<std::pair<double, int>> ready;
    auto node_ready = [&](int k) {
      for (int q = 0; q < n_first[k]; ++q) ready.push({prio[k], first_job[k] + q});
    };
    for (int k = 0; k < nt; ++k)
      if (waiting[k] == 0) node_ready(k);
    int remaining = nt;  // nodes not finished
    std::mutex mu;
    std::condition_variable cv;
    auto worker = [&]() {
      IlutWork W(n);
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [&] { return !ready.empty() || remaining == 0; });
        if (ready.empty()) return;
        const Job jb = jobs[ready.top().second];
        ready.pop();
        const int k = jb.node;
        const bool skip = poisoned[k] != 0;
        lk.unlock();
        if (!skip) {
          if (jb.kind == 0) {
            full_rows(k, W);
          } else if (jb.kind == 1) {
            for (int i = jb.r0; i < jb.r1; ++i) {
              const double thr = ilut_row_begin(A, tau, i, W);
              ilut_row_eliminate(i, thr, lo[k], node_of, rows, W);
              ilut_row_save(i, lo[k], thr, W, saved[k][i - lo[k]]);
            }
          } else {
            for (int i = lo[k]; i < hi[k]; ++i) {
              IlutRowState& R = saved[k][i - lo[k]];
              const double thr = ilut_row_restore(i, lo[k], R, W);
              R = IlutRowState();
              ilut_row_eliminate(i, thr, i, node_of, rows, W);
              if (!ilut_row_finish(i, thr, W, rows[k], &fail_st[k])) {
                fail_row[k] = i;
                break;
              }
            }
          }
        }
        lk.lock();
        bool node_done = jb.kind != 1;
        if (jb.kind == 1 && --p1_left[k] == 0) ready.push({prio[k], phase2[k]});
        if (node_done) {
          const int p = parent[k];
          if (p >= 0) {
            // a failed row leaves its ancestors unfactored (they would read it)
            if (skip || fail_row[k] >= 0) poisoned[p] = 1;
            if (--waiting[p] == 0) node_ready(p);
          }
          --remaining;
        }
        cv.notify_all();
      }
    };
    const int nthreads = std::min(host_threads(), nt);
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
  }
  // the first failing row in row order (rows before it do not depend on any
  // failing row, so it is the row a sequential pass stops at)
  int first = -1;
  gmg_status st = GMG_OK;
  for (int k = 0; k < nt; ++k)
    if (fail_row[k] >= 0 && (first < 0 || fail_row[k] < first)) { first = fail_row[k]; st = fail_st[k]; }
  if (first >= 0) return st;
  // concatenate the nodes' rows in row order
  std::vector<int> order(nt);
  for (int k = 0; k < nt; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return lo[x] < lo[y]; });
  std::vector<int64_t> loff(nt + 1, 0), uoff(nt + 1, 0);
  for (int q = 0; q < nt; ++q) {
    loff[q + 1] = loff[q] + (int64_t)rows[order[q]].lci.size();
    uoff[q + 1] = uoff[q] + (int64_t)rows[order[q]].uci.size();
  }
  if (loff[nt] > INT32_MAX || uoff[nt] > INT32_MAX) return GMG_ERR_OOM;  // int32 row pointers
  // the four entry arrays are sized (zero-filled, first-touched) by four
  // threads at once, then the nodes' rows are copied by all threads, each
  // node's own vectors released as soon as they are copied
  const int nthreads = std::min(host_threads(), nt);
  {
    auto sized = [&](int which) {
      switch (which) {
        case 0: L.ci.resize(loff[nt]); L.rp.assign(n + 1, 0); break;
        case 1: L.v.resize(loff[nt]); break;
        case 2: U.ci.resize(uoff[nt]); U.rp.assign(n + 1, 0); break;
        default: U.v.resize(uoff[nt]); break;
      }
    };
    if (nthreads >= 4) {
      std::vector<std::thread> pool;
      for (int w = 1; w < 4; ++w) pool.emplace_back(sized, w);
      sized(0);
      for (auto& t : pool) t.join();
    } else {
      for (int w = 0; w < 4; ++w) sized(w);
    }
  }
  auto copy_nodes = [&](int q0, int q1) {
    for (int q = q0; q < q1; ++q) {
      IlutNodeRows& R = rows[order[q]];
      const int nr = (int)R.lrp.size() - 1;
      for (int r = 0; r < nr; ++r) {
        L.rp[R.lo + r + 1] = (int)loff[q] + R.lrp[r + 1];
        U.rp[R.lo + r + 1] = (int)uoff[q] + R.urp[r + 1];
      }
      std::copy(R.lci.begin(), R.lci.end(), L.ci.begin() + loff[q]);
      std::copy(R.lv.begin(), R.lv.end(), L.v.begin() + loff[q]);
      std::copy(R.uci.begin(), R.uci.end(), U.ci.begin() + uoff[q]);
      std::copy(R.uv.begin(), R.uv.end(), U.v.begin() + uoff[q]);
      R = IlutNodeRows();
    }
  };
  if (nthreads <= 1) {
    copy_nodes(0, nt);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
      pool.emplace_back(copy_nodes, (int)((int64_t)nt * t / nthreads), (int)((int64_t)nt * (t + 1) / nthreads));
    for (auto& t : pool) t.join();
  }
  return GMG_OK;
}


// Nested-dissection numbering of the vertices of a symmetric graph (CSR
// without diagonal).  ND(S): at most 64 vertices -> ascending; disconnected
// -> its components in order of their smallest vertex, each by ND; otherwise
// BFS from min S, r = smallest vertex at the largest distance, d = distance
// from r inside S, L = max d (L < 2 -> ascending); m = smallest level holding
// at least half of S cumulatively, clamped to [1, L-1]; then ND(d < m),
// ND(d > m), and the separator d == m ascending.  Returns perm (position ->
// vertex).
std::vector<int> nd_numbering(int n, const std::vector<int>& rp_in, const std::vector<int>& ci_in,
                              std::vector<NdNode>* tree) {
  // A task owns a segment of seq (the vertices of one subgraph, ascending);
  // dissecting it stable-partitions the segment into [part a | part b |
  // separator] and hands the parts on as child tasks.  Taken depth first
  // (part a's subtree, then part b's, then the separator), the emitted order
  // is the final segment order itself, so disjoint segments can be dissected
  // concurrently and the numbering is seq once all tasks are done.  Tree
  // nodes are created under a lock and renumbered afterwards in the order a
  // depth-first pass creates them (both children of a node on its visit).
  struct Task { int kind, start, len, node; };  // kind 0: dissect, 1: emit as is
  struct Node { int lo = 0, hi = 0, parent = -1, a = -1, b = -1; };
  // small graphs are not worth the threads
  const int nthreads = n >= 4096 ? host_threads() : 1;
  // the neighbour lists without repeats (callers may list an edge from both
  // ends, and the traversal only needs each neighbour once)
  std::vector<int> rp(n + 1, 0), ci;
  {
    std::vector<int> cnt(n + 1, 0), tmp(ci_in.size());
    const int nt = std::max(1, std::min(nthreads, n / 4096));
    auto dedup = [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        int* b = tmp.data() + rp_in[i];
        std::copy(ci_in.begin() + rp_in[i], ci_in.begin() + rp_in[i + 1], b);
        std::sort(b, b + (rp_in[i + 1] - rp_in[i]));
        cnt[i + 1] = (int)(std::unique(b, b + (rp_in[i + 1] - rp_in[i])) - b);
      }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(dedup, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt));
    dedup(0, (int)((int64_t)n / nt));
    for (auto& th : pool) th.join();
    for (int i = 0; i < n; ++i) rp[i + 1] = rp[i] + cnt[i + 1];
    ci.resize(rp[n]);
    for (int i = 0; i < n; ++i) std::copy(tmp.begin() + rp_in[i], tmp.begin() + rp_in[i] + cnt[i + 1], ci.begin() + rp[i]);
  }
  std::vector<int> seq(n);
  for (int i = 0; i < n; ++i) seq[i] = i;
  // per vertex: the tag of the task that owns it (high 32 bits) and its BFS
  // distance + 1 in that task (low 32 bits, 0 = not reached), in one word so
  // a neighbour test touches one cache line
  std::unique_ptr<std::atomic<uint64_t>[]> mark(new std::atomic<uint64_t>[n > 0 ? n : 1]);
  for (int i = 0; i < n; ++i) mark[i].store(~0ull, std::memory_order_relaxed);
  auto dist_of = [&](int v) { return (int)(uint32_t)mark[v].load(std::memory_order_relaxed) - 1; };
  std::atomic<int> next_tag{0};
  std::vector<Node> nodes(1);
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Task> ready{{0, 0, n, 0}};
  int active = 0;

  // under mu: two children of node x
  auto children = [&](int x, int* na, int* nb) {
    *na = (int)nodes.size();
    *nb = *na + 1;
    nodes.resize(nodes.size() + 2);
    nodes[*na].parent = nodes[*nb].parent = x;
    nodes[x].a = *na;
    nodes[x].b = *nb;
  };

  // process one task; appends its child tasks to out (under no lock)
  auto run = [&](const Task& t, std::vector<int>& queue, std::vector<Task>& out, std::vector<int>& ids) {
    if (t.len == 0) return;
    int* b = seq.data() + t.start;
    int* e = b + t.len;
    if (t.kind == 1 || t.len <= 64) {
      // the node's own rows: numbered after all of its descendants'
      std::lock_guard<std::mutex> g(mu);
      nodes[t.node].lo = t.start;
      nodes[t.node].hi = t.start + t.len;
      return;
    }
    const uint64_t tag = (uint64_t)(uint32_t)next_tag.fetch_add(1, std::memory_order_relaxed) << 32;
    for (int* q = b; q != e; ++q) mark[*q].store(tag, std::memory_order_relaxed);
    auto bfs = [&](int src) {
      queue.clear();
      mark[src].store(tag | 1u, std::memory_order_relaxed);
      queue.push_back(src);
      for (size_t h = 0; h < queue.size(); ++h) {
        const int u = queue[h];
        const uint64_t du = (uint32_t)mark[u].load(std::memory_order_relaxed);  // distance + 1
        for (int p = rp[u]; p < rp[u + 1]; ++p) {
          const int v = ci[p];
          if (mark[v].load(std::memory_order_relaxed) == tag) {  // in the segment, not reached
            mark[v].store(tag | (du + 1), std::memory_order_relaxed);
            queue.push_back(v);
          }
        }
      }
    };
    bfs(*b);  // segments are kept ascending, so *b is the smallest vertex
    if ((int)queue.size() < t.len) {
      // disconnected: the component of *b, then the rest
      int* mid = std::stable_partition(b, e, [&](int v) { return dist_of(v) >= 0; });
      const int c0 = (int)(mid - b);
      {
        std::lock_guard<std::mutex> g(mu);
        children(t.node, &ids[0], &ids[1]);
      }
      out.push_back({0, t.start, c0, ids[0]});
      out.push_back({0, t.start + c0, t.len - c0, ids[1]});
      return;
    }
    int r = *b, far = 0;
    for (int* q = b; q != e; ++q) {
      const int d = dist_of(*q);
      if (d > far || (d == far && *q < r)) { far = d; r = *q; }
    }
    for (int* q = b; q != e; ++q) mark[*q].store(tag, std::memory_order_relaxed);
    bfs(r);
    std::vector<int>& dist = queue;  // the queue's job is done: reuse it for the distances in segment order
    dist.resize(t.len);
    int L = 0;
    for (int i = 0; i < t.len; ++i) {
      dist[i] = dist_of(b[i]);
      L = std::max(L, dist[i]);
    }
    if (L < 2) {
      out.push_back({1, t.start, t.len, t.node});
      return;
    }
    std::vector<int> cnt(L + 1, 0);
    for (int i = 0; i < t.len; ++i) cnt[dist[i]]++;
    int m = 0, cum = cnt[0];
    while (2.0 * cum < (double)t.len) cum += cnt[++m];
    m = std::min(std::max(m, 1), L - 1);
    int* m1 = std::stable_partition(b, e, [&](int v) { return dist_of(v) < m; });
    int* m2 = std::stable_partition(m1, e, [&](int v) { return dist_of(v) > m; });
    const int c0 = (int)(m1 - b), c1 = (int)(m2 - m1);
    {
      std::lock_guard<std::mutex> g(mu);
      children(t.node, &ids[0], &ids[1]);
    }
    out.push_back({0, t.start, c0, ids[0]});
    out.push_back({0, t.start + c0, c1, ids[1]});
    out.push_back({1, t.start + c0 + c1, t.len - c0 - c1, t.node});
  };

  constexpr int kLocalSubtree = 4096;
  auto worker = [&]() {
    std::vector<int> queue;
    std::vector<Task> out;
    std::vector<int> ids(2);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return !ready.empty() || active == 0; });
      if (ready.empty()) return;
      const Task t = ready.back();
      ready.pop_back();
      ++active;
      lk.unlock();
      out.clear();
      if (t.len <= kLocalSubtree) {
        // a small subtree: finished here, without the shared list
        std::vector<Task> local{t};
        while (!local.empty()) {
          const Task u = local.back();
          local.pop_back();
          const size_t o0 = out.size();
          run(u, queue, out, ids);
          local.insert(local.end(), out.begin() + o0, out.end());
          out.resize(o0);
        }
      } else {
        run(t, queue, out, ids);
      }
      lk.lock();
      ready.insert(ready.end(), out.begin(), out.end());
      --active;
      cv.notify_all();
    }
  };
  if (nthreads <= 1) {
    worker();
  } else {
    std::vector<std::thread> pool;
    for (int k = 0; k < nthreads; ++k) pool.emplace_back(worker);
    for (auto& th : pool) th.join();
  }
  if (tree) {
    // ids in depth-first creation order, then heights (children come after
    // their parent)
    const int nn = (int)nodes.size();
    std::vector<int> id(nn, -1), stack{0};
    id[0] = 0;
    int next = 1;
    while (!stack.empty()) {
      const int x = stack.back();
      stack.pop_back();
      if (nodes[x].a < 0) continue;
      id[nodes[x].a] = next++;
      id[nodes[x].b] = next++;
      stack.push_back(nodes[x].b);
      stack.push_back(nodes[x].a);
    }
    std::vector<NdNode> out(nn);
    for (int x = 0; x < nn; ++x)
      out[id[x]] = NdNode{nodes[x].lo, nodes[x].hi, nodes[x].parent >= 0 ? id[nodes[x].parent] : -1, 0};
    for (int k = nn - 1; k > 0; --k) {
      NdNode& p = out[out[k].parent];
      p.height = std::max(p.height, out[k].height + 1);
    }
    *tree = std::move(out);
  }
  return seq;
}

// Colour-class numbering: a greedy colouring in natural order (vertex i
// takes the smallest colour no neighbour j < i has), then the vertices by
// colour, ascending within a colour.  rp/ci: the symmetric neighbour lists
// (repeats allowed).
std::vector<int> color_numbering(int n, const std::vector<int>& rp, const std::vector<int>& ci) {
  std::vector<int> color(n), last(n + 1, -1);
  int ncol = 0;
  for (int i = 0; i < n; ++i) {
    for (int q = rp[i]; q < rp[i + 1]; ++q)
      if (ci[q] < i) last[color[ci[q]]] = i;
    int c = 0;
    while (last[c] == i) ++c;
    color[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  std::vector<int> start(ncol + 1, 0), perm(n);
  for (int i = 0; i < n; ++i) start[color[i] + 1]++;
  for (int c = 0; c < ncol; ++c) start[c + 1] += start[c];
  for (int i = 0; i < n; ++i) perm[start[color[i]]++] = i;
  return perm;
}

// Sparse approximate inverse of A (square host CSR) with A's pattern: column
// j of M minimises ||A m - e_j||_2 over m supported on column j's pattern J.
// The rows that those columns reach form a small dense least-squares
// problem, solved by Householder QR (column-major, the reflector kept in the
// column it annihilates) and back substitution.  Columns are independent and
// spread over the host threads in blocks.
gmg_status host_spai(const HCsr& A, HCsr& M) {
  const int n = A.n;
  const size_t nnz = A.ci.size();
  // column access: cp/cr/cv list column j's rows ascending, csrc the entry in A
  std::vector<int> cp(n + 1, 0), cr(nnz), csrc(nnz);
  std::vector<double> cv(nnz);
  for (size_t q = 0; q < nnz; ++q) cp[A.ci[q] + 1]++;
  for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
  {
    std::vector<int> at(cp.begin(), cp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int q = A.rp[i]; q < A.rp[i + 1]; ++q) {
        const int k = at[A.ci[q]]++;
        cr[k] = i;
        cv[k] = A.v[q];
        csrc[k] = q;
      }
  }
  M.n = n;
  M.rp = A.rp;
  M.ci = A.ci;
  M.v.assign(nnz, 0.0);
  constexpr int kBlock = 256;
  std::atomic<int> next{0};
  std::atomic<int> status{GMG_OK};
  auto work = [&]() {
    std::vector<int> slot(n, -1), rows;
    std::vector<double> H, b, m;
    for (;;) {
      const int j0 = next.fetch_add(kBlock);
      if (j0 >= n || status.load(std::memory_order_relaxed) != GMG_OK) return;
      for (int j = j0; j < std::min(n, j0 + kBlock); ++j) {
        const int nj = cp[j + 1] - cp[j];
        const int* J = cr.data() + cp[j];
        rows.clear();
        for (int c = 0; c < nj; ++c)
          for (int q = cp[J[c]]; q < cp[J[c] + 1]; ++q)
            if (slot[cr[q]] < 0) { slot[cr[q]] = 0; rows.push_back(cr[q]); }
        std::sort(rows.begin(), rows.end());
        const int ni = (int)rows.size();
        for (int r = 0; r < ni; ++r) slot[rows[r]] = r;
        H.assign((size_t)ni * nj, 0.0);
        for (int c = 0; c < nj; ++c)
          for (int q = cp[J[c]]; q < cp[J[c] + 1]; ++q) H[(size_t)c * ni + slot[cr[q]]] = cv[q];
        b.assign(ni, 0.0);
        if (slot[j] >= 0) b[slot[j]] = 1.0;
        gmg_status st = GMG_OK;
        for (int c = 0; c < nj && c < ni && st == GMG_OK; ++c) {
          double* x = &H[(size_t)c * ni];
          double ss = 0.0;
          for (int r = c; r < ni; ++r) ss += x[r] * x[r];
          const double nrm = std::sqrt(ss);
          if (nrm == 0.0) { st = GMG_ERR_ZERO_PIVOT; break; }
          const double alpha = x[c] >= 0.0 ? -nrm : nrm;
          x[c] -= alpha;
          double vv = 0.0;
          for (int r = c; r < ni; ++r) vv += x[r] * x[r];
          auto reflect = [&](double* y) {
            double d = 0.0;
            for (int r = c; r < ni; ++r) d += x[r] * y[r];
            const double f = 2.0 * d / vv;
            for (int r = c; r < ni; ++r) y[r] -= f * x[r];
          };
          for (int k = c + 1; k < nj; ++k) reflect(&H[(size_t)k * ni]);
          reflect(b.data());
          x[c] = alpha;
        }
        if (st == GMG_OK && ni < nj) st = GMG_ERR_ZERO_PIVOT;
        m.assign(nj, 0.0);
        for (int c = nj - 1; c >= 0 && st == GMG_OK; --c) {
          double t = b[c];
          for (int k = c + 1; k < nj; ++k) t -= H[(size_t)k * ni + c] * m[k];
          m[c] = t / H[(size_t)c * ni + c];
          if (!std::isfinite(m[c])) st = GMG_ERR_NONFINITE;
        }
        for (int r = 0; r < ni; ++r) slot[rows[r]] = -1;
        if (st != GMG_OK) {
          int expect = GMG_OK;
          status.compare_exchange_strong(expect, st);
          return;
        }
        // M(J[c], j) sits where A(J[c], j) does
        for (int c = 0; c < nj; ++c) M.v[csrc[cp[j] + c]] = m[c];
      }
    }
  };
  const int nt = std::max(1, std::min(host_threads(), (n + kBlock - 1) / kBlock));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  return (gmg_status)status.load();
}

}  // namespace gmg
