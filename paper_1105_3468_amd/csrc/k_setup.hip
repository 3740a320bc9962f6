// Setup kernels: the symmetric weighted graph of A, multi-pass handshake
// matching, canonical aggregate numbering, the aggregate graph and the
// Galerkin product A_c = P^T A P.
//
// The aggregates and A_c are reproducible bit for bit: matching decisions use
// a strict total order on edges (quantised weight, then a SplitMix64 hash of
// the end points, then the end points), and every floating-point sum is taken
// in the order of the fine CSR entries (members ascending, then columns
// ascending), using additions only.
#include "gmg_internal.h"
#include "kcommon.h"

namespace gmg {

static unsigned g1(int64_t n, unsigned bs = 256) {
  int64_t g = (n + bs - 1) / bs;
  return (unsigned)(g < 1 ? 1 : g);
}

// ----------------------------------------------------------- weighted graph
// Row i of G0 merges row i of A and row i of A^T (both column-sorted):
// an edge j != i exists if either is stored, w = |a_ij| + |a_ji|.
template <bool FILL>
__global__ void k_graph(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                        const double* __restrict__ v, const int* __restrict__ trp,
                        const int* __restrict__ tci, const double* __restrict__ tv,
                        int* __restrict__ cnt, const int* __restrict__ grp, int* __restrict__ gci,
                        double* __restrict__ gw) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = rp[i], pe = rp[i + 1], q = trp[i], qe = trp[i + 1];
  int c = 0, o = FILL ? grp[i] : 0;
  while (p < pe || q < qe) {
    const int cp = p < pe ? ci[p] : n, cq = q < qe ? tci[q] : n;
    const int j = cp < cq ? cp : cq;
    double aij = 0.0, aji = 0.0;
    if (cp == j) { aij = v[p]; ++p; }
    if (cq == j) { aji = tv[q]; ++q; }
    if (j == i) continue;
    if (FILL) {
      gci[o + c] = j;
      gw[o + c] = fabs(aij) + fabs(aji);
    }
    ++c;
  }
  if (!FILL) cnt[i] = c;
}

void build_graph(int n, const int* rp, const int* ci, const double* v, const int* trp, const int* tci,
                 const double* tv, DBuf<int>& grp, DBuf<int>& gci, DBuf<double>& gw, hipStream_t s) {
  DBuf<int> cnt, tmp;
  cnt.alloc((size_t)n + 1);
  grp.alloc((size_t)n + 1);
  launch_fill_u32(reinterpret_cast<unsigned*>(cnt.p), 0u, (size_t)n + 1, s);
  hipLaunchKernelGGL(k_graph<false>, dim3(g1(n)), dim3(256), 0, s, n, rp, ci, v, trp, tci, tv, cnt.p,
                     (const int*)nullptr, (int*)nullptr, (double*)nullptr);
  launch_exclusive_scan_int(cnt.p, grp.p, n + 1, s, tmp);
  int nnz = 0;
  d2h(&nnz, grp.p + n, 1, s);
  HIPCK(hipStreamSynchronize(s));
  gci.alloc(nnz > 0 ? nnz : 1);
  gw.alloc(nnz > 0 ? nnz : 1);
  hipLaunchKernelGGL(k_graph<true>, dim3(g1(n)), dim3(256), 0, s, n, rp, ci, v, trp, tci, tv, cnt.p, grp.p,
                     gci.p, gw.p);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(s));
}

// --------------------------------------------------------------- edge keys
__device__ __forceinline__ uint64_t sm64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

struct Key {
  uint64_t q, h;
  int lo, hi;
};

__device__ __forceinline__ Key edge_key(double w, int a, int b, int qbits, uint64_t seed) {
  Key k;
  k.q = __builtin_bit_cast(uint64_t, w) >> (52 - qbits);
  k.lo = a < b ? a : b;
  k.hi = a < b ? b : a;
  k.h = sm64_out(((uint64_t)(uint32_t)k.lo << 32 | (uint64_t)(uint32_t)k.hi) ^ seed);
  return k;
}
__device__ __forceinline__ bool key_gt(const Key& x, const Key& y) {
  if (x.q != y.q) return x.q > y.q;
  if (x.h != y.h) return x.h > y.h;
  if (x.lo != y.lo) return x.lo > y.lo;
  return x.hi > y.hi;
}

// every unmatched vertex points at its best unmatched neighbour
__global__ void k_cand(int nv, const int* __restrict__ rp, const int* __restrict__ ci,
                       const double* __restrict__ w, const int* __restrict__ mate, int* __restrict__ cand,
                       int qbits, uint64_t seed, int* any) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int best = -1;
  Key bk = {0, 0, 0, 0};
  if (mate[v] < 0) {
    for (int p = rp[v]; p < rp[v + 1]; ++p) {
      const int u = ci[p];
      if (u == v || mate[u] >= 0) continue;
      const Key k = edge_key(w[p], v, u, qbits, seed);
      if (best < 0 || key_gt(k, bk)) { bk = k; best = u; }
    }
  }
  cand[v] = best;
  if (best >= 0) *any = 1;   // benign race: every writer stores 1
}

// mutual pointers become matched pairs
__global__ void k_mutual(int nv, const int* __restrict__ cand, int* __restrict__ mate) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int u = cand[v];
  if (u >= 0 && cand[u] == v) mate[v] = u;
}

__global__ void k_leader(int nv, const int* __restrict__ mate, int* __restrict__ flag) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v > nv) return;
  flag[v] = (v < nv && (mate[v] < 0 || v < mate[v])) ? 1 : 0;
}
// after the scan nid[v] holds the rank of leader v; followers copy their mate's
__global__ void k_follow(int nv, const int* __restrict__ mate, int* __restrict__ nid) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int u = mate[v];
  if (u >= 0 && u < v) nid[v] = nid[u];
}
__global__ void k_compose(int n, int* __restrict__ agg, const int* __restrict__ nid) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) agg[k] = nid[agg[k]];
}
__global__ void k_iota(int n, int* a) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = k;
}

// ---------------------------------------------------------------- members
__global__ void k_count_agg(int n, const int* __restrict__ agg, int* __restrict__ cnt) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) atomicAdd(&cnt[agg[k]], 1);
}
__global__ void k_scatter_mem(int n, const int* __restrict__ agg, int* __restrict__ fill, int* __restrict__ amem) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) amem[atomicAdd(&fill[agg[k]], 1)] = k;
}
__global__ void k_sort_seg(int m, const int* __restrict__ ptr, int* __restrict__ a) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= m) return;
  const int s = ptr[I], e = ptr[I + 1];
  for (int p = s + 1; p < e; ++p) {
    const int key = a[p];
    int q = p - 1;
    while (q >= s && a[q] > key) { a[q + 1] = a[q]; --q; }
    a[q + 1] = key;
  }
}

void build_members(int n, int nc, const int* agg, DBuf<int>& aptr, DBuf<int>& amem, hipStream_t s) {
  DBuf<int> cnt, tmp, fill;
  cnt.alloc((size_t)nc + 1);
  aptr.alloc((size_t)nc + 1);
  amem.alloc(n > 0 ? n : 1);
  fill.alloc((size_t)nc + 1);
  launch_fill_u32(reinterpret_cast<unsigned*>(cnt.p), 0u, (size_t)nc + 1, s);
  hipLaunchKernelGGL(k_count_agg, dim3(g1(n)), dim3(256), 0, s, n, agg, cnt.p);
  launch_exclusive_scan_int(cnt.p, aptr.p, nc + 1, s, tmp);
  d2d(fill.p, aptr.p, (size_t)nc + 1, s);
  hipLaunchKernelGGL(k_scatter_mem, dim3(g1(n)), dim3(256), 0, s, n, agg, fill.p, amem.p);
  hipLaunchKernelGGL(k_sort_seg, dim3(g1(nc)), dim3(256), 0, s, nc, aptr.p, amem.p);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(s));
}

// ------------------------------------------- aggregated matrices and graphs
// For aggregate I, visit fine entries (k, l) with k in G_I (members ascending)
// and l ascending; keep J = agg[l] when UPPER_ONLY is false or J > I.
template <bool UPPER_ONLY>
__global__ void k_agg_count(int nc, const int* __restrict__ aptr, const int* __restrict__ amem,
                            const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ agg,
                            int* __restrict__ cnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int c = 0;
  for (int m = aptr[I]; m < aptr[I + 1]; ++m) {
    const int k = amem[m];
    for (int p = rp[k]; p < rp[k + 1]; ++p)
      if (!UPPER_ONLY || agg[ci[p]] > I) ++c;
  }
  cnt[I] = c;
}

// Fill the raw (J, value) list of aggregate I in visiting order, sort it
// stably by J (insertion sort keeps equal J in visiting order), add runs of
// equal J front to back, and leave the compacted list at the segment start.
template <bool UPPER_ONLY>
__global__ void k_agg_fill(int nc, const int* __restrict__ aptr, const int* __restrict__ amem,
                           const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                           const int* __restrict__ agg, const int* __restrict__ off, int* __restrict__ rj,
                           double* __restrict__ rv, int* __restrict__ dcnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int s = off[I];
  int e = s;
  for (int m = aptr[I]; m < aptr[I + 1]; ++m) {
    const int k = amem[m];
    for (int p = rp[k]; p < rp[k + 1]; ++p) {
      const int J = agg[ci[p]];
      if (UPPER_ONLY && J <= I) continue;
      rj[e] = J;
      rv[e] = v[p];
      ++e;
    }
  }
  for (int p = s + 1; p < e; ++p) {
    const int kj = rj[p];
    const double kv = rv[p];
    int q = p - 1;
    while (q >= s && rj[q] > kj) { rj[q + 1] = rj[q]; rv[q + 1] = rv[q]; --q; }
    rj[q + 1] = kj;
    rv[q + 1] = kv;
  }
  int o = s;
  int p = s;
  while (p < e) {
    const int J = rj[p];
    double sum = rv[p];
    int q = p + 1;
    while (q < e && rj[q] == J) { sum = sum + rv[q]; ++q; }
    rj[o] = J;
    rv[o] = sum;
    ++o;
    p = q;
  }
  dcnt[I] = o - s;
}

__global__ void k_compact(int nc, const int* __restrict__ off, const int* __restrict__ dst_rp,
                          const int* __restrict__ rj, const double* __restrict__ rv, int* __restrict__ cj,
                          double* __restrict__ cv) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int s = off[I], d = dst_rp[I], c = dst_rp[I + 1] - d;
  for (int t = 0; t < c; ++t) {
    cj[d + t] = rj[s + t];
    cv[d + t] = rv[s + t];
  }
}

// Aggregated CSR (nc rows) from fine CSR (rp, ci, v) and the aggregates.
template <bool UPPER_ONLY>
static void aggregate_csr(int nc, const int* aptr, const int* amem, const int* rp, const int* ci, const double* v,
                          const int* agg, DBuf<int>& orp, DBuf<int>& oci, DBuf<double>& ov, int64_t* onnz,
                          hipStream_t s) {
  DBuf<int> cnt, off, dcnt, tmp, rj;
  DBuf<double> rv;
  cnt.alloc((size_t)nc + 1);
  off.alloc((size_t)nc + 1);
  dcnt.alloc((size_t)nc + 1);
  launch_fill_u32(reinterpret_cast<unsigned*>(cnt.p), 0u, (size_t)nc + 1, s);
  launch_fill_u32(reinterpret_cast<unsigned*>(dcnt.p), 0u, (size_t)nc + 1, s);
  hipLaunchKernelGGL(k_agg_count<UPPER_ONLY>, dim3(g1(nc)), dim3(256), 0, s, nc, aptr, amem, rp, ci, agg, cnt.p);
  launch_exclusive_scan_int(cnt.p, off.p, nc + 1, s, tmp);
  int raw = 0;
  d2h(&raw, off.p + nc, 1, s);
  HIPCK(hipStreamSynchronize(s));
  rj.alloc(raw > 0 ? raw : 1);
  rv.alloc(raw > 0 ? raw : 1);
  hipLaunchKernelGGL(k_agg_fill<UPPER_ONLY>, dim3(g1(nc, 128)), dim3(128), 0, s, nc, aptr, amem, rp, ci, v, agg,
                     off.p, rj.p, rv.p, dcnt.p);
  orp.alloc((size_t)nc + 1);
  launch_exclusive_scan_int(dcnt.p, orp.p, nc + 1, s, tmp);
  int nnz = 0;
  d2h(&nnz, orp.p + nc, 1, s);
  HIPCK(hipStreamSynchronize(s));
  oci.alloc(nnz > 0 ? nnz : 1);
  ov.alloc(nnz > 0 ? nnz : 1);
  hipLaunchKernelGGL(k_compact, dim3(g1(nc)), dim3(256), 0, s, nc, off.p, orp.p, rj.p, rv.p, oci.p, ov.p);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(s));
  *onnz = nnz;
}

// row I of the merged graph: transposed (lower) part, then the upper part
template <bool FILL>
__global__ void k_merge_sym(int nv, const int* __restrict__ lrp, const int* __restrict__ lci,
                            const double* __restrict__ lv, const int* __restrict__ urp,
                            const int* __restrict__ uci, const double* __restrict__ uv, int* __restrict__ cnt,
                            const int* __restrict__ grp, int* __restrict__ gci, double* __restrict__ gw) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nv) return;
  const int nl = lrp[I + 1] - lrp[I], nu = urp[I + 1] - urp[I];
  if (!FILL) { cnt[I] = nl + nu; return; }
  int o = grp[I];
  for (int t = 0; t < nl; ++t) { gci[o] = lci[lrp[I] + t]; gw[o] = lv[lrp[I] + t]; ++o; }
  for (int t = 0; t < nu; ++t) { gci[o] = uci[urp[I] + t]; gw[o] = uv[urp[I] + t]; ++o; }
}

int aggregate(int n, const DBuf<int>& grp0, const DBuf<int>& gci0, const DBuf<double>& gw0, double cf,
              int max_passes, int qbits, uint64_t seed, DBuf<int>& agg, int* passes_out, int* rounds_out,
              hipStream_t s) {
  agg.alloc(n > 0 ? n : 1);
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(g1(n)), dim3(256), 0, s, n, agg.p);
  int nv = n;
  const long target = (long)std::floor((double)n / cf);
  int passes = 0, rounds_total = 0;
  DBuf<int> mate, cand, nid, flag, any, tmp;
  mate.alloc(n + 1);
  cand.alloc(n + 1);
  nid.alloc(n + 2);
  flag.alloc(n + 2);
  any.alloc(1);
  // current graph (pass 1: G0)
  DBuf<int> crp, cci;
  DBuf<double> cw;
  const int *rp = grp0.p, *ci = gci0.p;
  const double* w = gw0.p;
  int* hbuf = nullptr;
  HIPCK(hipHostMalloc(&hbuf, sizeof(int) * 2, hipHostMallocDefault));
  struct HostFree { int* p; ~HostFree() { if (p) (void)hipHostFree(p); } } hf{hbuf};
  while (nv > target && passes < max_passes) {
    launch_fill_u32(reinterpret_cast<unsigned*>(mate.p), 0xFFFFFFFFu, (size_t)nv, s);
    int rounds = 0;
    for (;;) {
      launch_fill_u32(reinterpret_cast<unsigned*>(any.p), 0u, 1, s);
      hipLaunchKernelGGL(k_cand, dim3(g1(nv)), dim3(256), 0, s, nv, rp, ci, w, mate.p, cand.p, qbits, seed, any.p);
      HIPCK(hipGetLastError());
      d2h(hbuf, any.p, 1, s);
      HIPCK(hipStreamSynchronize(s));
      if (!hbuf[0]) break;
      ++rounds;
      if (rounds > 4 * 1024 * 1024) fail(GMG_ERR_HIP, "matching did not terminate");
      hipLaunchKernelGGL(k_mutual, dim3(g1(nv)), dim3(256), 0, s, nv, cand.p, mate.p);
      HIPCK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_leader, dim3(g1(nv + 1)), dim3(256), 0, s, nv, mate.p, flag.p);
    launch_exclusive_scan_int(flag.p, nid.p, nv + 1, s, tmp);
    hipLaunchKernelGGL(k_follow, dim3(g1(nv)), dim3(256), 0, s, nv, mate.p, nid.p);
    HIPCK(hipGetLastError());
    d2h(hbuf, nid.p + nv, 1, s);
    HIPCK(hipStreamSynchronize(s));
    const int cnt = hbuf[0];
    if (cnt == nv) break;  // no pair matched
    ++passes;
    rounds_total += rounds;
    hipLaunchKernelGGL(k_compose, dim3(g1(n)), dim3(256), 0, s, n, agg.p, nid.p);
    HIPCK(hipGetLastError());
    nv = cnt;
    if (!(nv > target && passes < max_passes)) break;  // no further pass needs a graph
    // aggregate graph: w_IJ (I < J) summed in fine CSR order, mirrored
    DBuf<int> aptr, amem, urp, uci, lrp, lci, nrp, ncnt;
    DBuf<double> uv, lv;
    build_members(n, nv, agg.p, aptr, amem, s);
    int64_t nu = 0;
    aggregate_csr<true>(nv, aptr.p, amem.p, grp0.p, gci0.p, gw0.p, agg.p, urp, uci, uv, &nu, s);
    transpose_csr(nv, nv, nu, urp.p, uci.p, uv.p, lrp, lci, &lv, nullptr, s);
    ncnt.alloc((size_t)nv + 1);
    nrp.alloc((size_t)nv + 1);
    launch_fill_u32(reinterpret_cast<unsigned*>(ncnt.p), 0u, (size_t)nv + 1, s);
    hipLaunchKernelGGL(k_merge_sym<false>, dim3(g1(nv)), dim3(256), 0, s, nv, lrp.p, lci.p, lv.p, urp.p, uci.p, uv.p,
                       ncnt.p, (const int*)nullptr, (int*)nullptr, (double*)nullptr);
    launch_exclusive_scan_int(ncnt.p, nrp.p, nv + 1, s, tmp);
    DBuf<int> ngci;
    DBuf<double> ngw;
    ngci.alloc(2 * nu > 0 ? 2 * nu : 1);
    ngw.alloc(2 * nu > 0 ? 2 * nu : 1);
    hipLaunchKernelGGL(k_merge_sym<true>, dim3(g1(nv)), dim3(256), 0, s, nv, lrp.p, lci.p, lv.p, urp.p, uci.p, uv.p,
                       ncnt.p, nrp.p, ngci.p, ngw.p);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    crp = std::move(nrp);
    cci = std::move(ngci);
    cw = std::move(ngw);
    rp = crp.p;
    ci = cci.p;
    w = cw.p;
  }
  HIPCK(hipStreamSynchronize(s));
  *passes_out = passes;
  *rounds_out = rounds_total;
  return nv;
}

void relabel(int n, int* agg, const int* rank, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_compose, dim3(g1(n)), dim3(256), 0, s, n, agg, rank);
  HIPCK(hipGetLastError());
}

void galerkin(int n, int nc, const int* rp, const int* ci, const double* v, const int* agg, const int* aptr,
              const int* amem, DCsr& Ac, hipStream_t s) {
  (void)n;
  Ac.n = nc;
  Ac.m = nc;
  aggregate_csr<false>(nc, aptr, amem, rp, ci, v, agg, Ac.rp, Ac.ci, Ac.v, &Ac.nnz, s);
}

}  // namespace gmg
