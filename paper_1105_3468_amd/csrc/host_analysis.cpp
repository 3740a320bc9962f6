// Host-side analysis steps of the setup: dependency-level schedules of the
// triangular factors, and the row-wise ILUT factorisation of the coarse matrix.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
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
gmg_status host_ilut(const HCsr& A, double tau, HCsr& L, HCsr& U) {
  const int n = A.n;
  L.n = U.n = n;
  L.rp.assign(n + 1, 0);
  U.rp.assign(n + 1, 0);
  L.ci.clear(); L.v.clear(); U.ci.clear(); U.v.clear();
  L.ci.reserve(A.ci.size()); L.v.reserve(A.ci.size());
  U.ci.reserve(A.ci.size()); U.v.reserve(A.ci.size());
  std::vector<double> w(n > 0 ? n : 1, 0.0);
  std::vector<signed char> state(n > 0 ? n : 1, 0);  // 0 absent, 1 present, 2 dropped
  std::vector<int> touched;
  touched.reserve(256);
  std::priority_queue<int, std::vector<int>, std::greater<int>> pending;
  for (int i = 0; i < n; ++i) {
    double ss = 0.0;
    touched.clear();
    for (int p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int j = A.ci[p];
      ss = ss + A.v[p] * A.v[p];
      w[j] = A.v[p];
      state[j] = 1;
      touched.push_back(j);
      if (j < i) pending.push(j);
    }
    const double thr = tau * std::sqrt(ss);
    if (state[i] == 0) { state[i] = 1; w[i] = 0.0; touched.push_back(i); }
    while (!pending.empty()) {
      const int k = pending.top();
      pending.pop();
      if (std::fabs(w[k]) < thr) { w[k] = 0.0; state[k] = 2; continue; }
      const int uk = U.rp[k];
      const double lik = w[k] / U.v[uk];
      w[k] = lik;
      for (int r = uk + 1; r < U.rp[k + 1]; ++r) {
        const int j = U.ci[r];
        if (state[j] == 0) {
          state[j] = 1;
          w[j] = 0.0;
          touched.push_back(j);
          if (j < i) pending.push(j);
        }
        w[j] = w[j] - lik * U.v[r];
      }
    }
    std::sort(touched.begin(), touched.end());
    const double d = w[i];
    U.ci.push_back(i);
    U.v.push_back(d);
    for (int j : touched) {
      if (j < i) {
        if (state[j] == 1) { L.ci.push_back(j); L.v.push_back(w[j]); }
      } else if (j > i) {
        if (!(std::fabs(w[j]) < thr)) { U.ci.push_back(j); U.v.push_back(w[j]); }
      }
      state[j] = 0;
      w[j] = 0.0;
    }
    L.rp[i + 1] = (int)L.ci.size();
    U.rp[i + 1] = (int)U.ci.size();
    if (d == 0.0) return GMG_ERR_ZERO_PIVOT;
    if (!std::isfinite(d)) return GMG_ERR_NONFINITE;
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
std::vector<int> nd_numbering(int n, const std::vector<int>& rp, const std::vector<int>& ci) {
  struct Task { int kind, start, len; };  // kind 0: dissect, 1: emit as is
  std::vector<int> seq(n), perm;
  perm.reserve(n);
  for (int i = 0; i < n; ++i) seq[i] = i;
  std::vector<int> mark(n, -1), dist(n, -1), queue;
  queue.reserve(n);
  std::vector<Task> stack{{0, 0, n}};
  int tag = 0;
  auto bfs = [&](int src) {
    queue.clear();
    dist[src] = 0;
    queue.push_back(src);
    for (size_t h = 0; h < queue.size(); ++h) {
      const int u = queue[h];
      for (int p = rp[u]; p < rp[u + 1]; ++p) {
        const int v = ci[p];
        if (mark[v] == tag && dist[v] < 0) {
          dist[v] = dist[u] + 1;
          queue.push_back(v);
        }
      }
    }
  };
  while (!stack.empty()) {
    const Task t = stack.back();
    stack.pop_back();
    if (t.len == 0) continue;
    int* b = seq.data() + t.start;
    int* e = b + t.len;
    if (t.kind == 1 || t.len <= 64) {
      perm.insert(perm.end(), b, e);
      continue;
    }
    ++tag;
    for (int* q = b; q != e; ++q) { mark[*q] = tag; dist[*q] = -1; }
    bfs(*b);  // segments are kept ascending, so *b is the smallest vertex
    if ((int)queue.size() < t.len) {
      int* mid = std::stable_partition(b, e, [&](int v) { return dist[v] >= 0; });
      const int c0 = (int)(mid - b);
      stack.push_back({0, t.start + c0, t.len - c0});
      stack.push_back({0, t.start, c0});
      continue;
    }
    int r = *b, far = 0;
    for (int* q = b; q != e; ++q)
      if (dist[*q] > far || (dist[*q] == far && *q < r)) { far = dist[*q]; r = *q; }
    for (int* q = b; q != e; ++q) dist[*q] = -1;
    bfs(r);
    int L = 0;
    for (int* q = b; q != e; ++q) L = std::max(L, dist[*q]);
    if (L < 2) {
      stack.push_back({1, t.start, t.len});
      continue;
    }
    std::vector<int> cnt(L + 1, 0);
    for (int* q = b; q != e; ++q) cnt[dist[*q]]++;
    int m = 0, cum = cnt[0];
    while (2.0 * cum < (double)t.len) cum += cnt[++m];
    m = std::min(std::max(m, 1), L - 1);
    int* m1 = std::stable_partition(b, e, [&](int v) { return dist[v] < m; });
    int* m2 = std::stable_partition(m1, e, [&](int v) { return dist[v] > m; });
    const int c0 = (int)(m1 - b), c1 = (int)(m2 - m1);
    stack.push_back({1, t.start + c0 + c1, t.len - c0 - c1});
    stack.push_back({0, t.start + c0, c1});
    stack.push_back({0, t.start, c0});
  }
  return perm;
}

}  // namespace gmg
