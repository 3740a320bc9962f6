/*
 * gmg_oracle.c -- TEST INFRASTRUCTURE ONLY (never part of the product path).
 *
 * Plain, sequential, FP64 reference of the two-grid matching-aggregation AMG
 * preconditioner inside flexible GMRES, written from the paper
 * (Kumar, "Aggregation based on graph matching and inexact coarse grid solve
 * for algebraic multigrid"):
 *
 *   aggregates G_i and boolean P ................ Section 2, Eq. (interp), Eq. (aggr)
 *   coarse operator A_c = P^T A P ................ Section 2, Eq. (E:galerkin) and the
 *                                                  double-sum formula after Eq. (aggr)
 *   smoother S = L0 U0 = ILU(0)(A) ............... Section 2 (choice of S), Algorithm 1 setup
 *   ... or ILU(0) of A in nested-dissection order  the GMG-ND variant (Section 3.1 variant
 *       (S = Q^T L0 U0 Q) .......................  list and the comments on ND ordering)
 *   ... or in colour-class order (multicolour) .. a reading of the same comments: any
 *                                                  reordering that lets ILU(0) run in parallel
 *   inexact coarse factors ILUT(A_c) ............. Section 2 (ILU(t) paragraph), Algorithm 1 setup
 *   two-grid preconditioner B~ ................... Eq. (twogrid) and Algorithm 1 "SOLVE B~q=z",
 *                                                  "SOLVE M~g=h"
 *   Krylov accelerator ........................... Algorithm 1 (GMRES with Givens rotations)
 *
 * Where the paper uses a graph partitioner the oracle uses deterministic
 * handshake (locally dominant edge) matching, several passes, with a strict
 * total order on edges; the paper's GMRES is taken right-preconditioned and
 * flexible (FGMRES), which allows a preconditioner evaluated in FP32.
 *
 * Only tests, the package smoke check and the benchmark's CPU-baseline leg
 * load this file.  It shares no code with the HIP library.
 * Built with: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_ERR_INVALID (-1)
#define OR_ERR_OOM (-3)
#define OR_ERR_ZERO_PIVOT (-4)
#define OR_ERR_BREAKDOWN (-5)
#define OR_ERR_NONFINITE (-6)

typedef struct {
    double cf;           /* coarsening factor N / N_c (target)                  */
    int max_passes;      /* matching passes at most                               */
    int qbits;           /* mantissa bits of the weight kept in the edge key      */
    uint64_t seed;       /* hash seed of the edge key                             */
    double ilut_tau;     /* ILUT drop tolerance (relative to the row 2-norm)      */
    int coarse_mode;     /* 0: exact triangular sweeps, 1: Jacobi sweeps,
                            2: sparse approximate inverse of A_c                 */
    int coarse_sweeps;   /* Jacobi sweeps per factor when coarse_mode == 1        */
    int coarse_order;    /* 0: aggregates by smallest fine index; 1: nested dissection */
    int fine_order;      /* 0: ILU(0) smoother on A's numbering; 1: on A renumbered by
                            nested dissection (the GMG-ND variant); 2: by colour
                            classes of a greedy colouring (multicolour ILU(0))      */
} or_opts;

typedef struct {
    int n;
    int *rp, *ci;
    double *v;
} csr_t;

typedef struct {
    csr_t A;             /* fine matrix (copy)                          */
    csr_t G;             /* symmetric weighted graph of A               */
    int nc;              /* number of aggregates                        */
    int *agg;            /* fine index -> aggregate                     */
    int *aptr, *amem;    /* aggregate member lists, ascending           */
    int passes, rounds;
    csr_t Ac;            /* coarse matrix                               */
    csr_t F;             /* the smoother's matrix: A (fine_order 0) or  */
                         /* Q A Q^T with (Q x)_k = x_{fperm[k]}          */
    int *fperm;          /* position -> fine unknown (fine_order 1)     */
    double *ilu;         /* ILU(0) values on F's pattern                */
    int *dpos;           /* position of the diagonal in each row of F   */
    csr_t Mc;            /* sparse approximate inverse of A_c (coarse_mode 2)    */
    csr_t Lc, Uc;        /* ILUT factors: Lc strictly lower (unit diag implied),
                            Uc upper with the diagonal stored first    */
    or_opts o;
    /* FP32 copies for the single-precision preconditioner */
    float *v32, *ilu32, *lc32, *uc32, *mc32;
} or_solver;

static void csr_free(csr_t *m) {
    free(m->rp); free(m->ci); free(m->v);
    m->rp = NULL; m->ci = NULL; m->v = NULL;
}

/* ------------------------------------------------------------------------ */
/* Edge key: (Q(w), H(lo, hi), lo, hi), larger wins.                         */
/* Q keeps the exponent and the top qbits mantissa bits of a weight w >= 0.  */
/* H is the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).    */
/* ------------------------------------------------------------------------ */
static uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t q, h; int lo, hi; } ekey;

static ekey make_key(double w, int a, int b, int qbits, uint64_t seed) {
    ekey k;
    uint64_t bits;
    memcpy(&bits, &w, 8);
    k.q = bits >> (52 - qbits);
    k.lo = a < b ? a : b;
    k.hi = a < b ? b : a;
    k.h = sm64_mix((((uint64_t)(uint32_t)k.lo << 32) | (uint64_t)(uint32_t)k.hi) ^ seed);
    return k;
}

/* 1 if x beats y */
static int key_greater(const ekey *x, const ekey *y) {
    if (x->q != y->q) return x->q > y->q;
    if (x->h != y->h) return x->h > y->h;
    if (x->lo != y->lo) return x->lo > y->lo;
    return x->hi > y->hi;
}

/* ------------------------------------------------------------------------ */
/* Symmetric weighted graph: edge {i,j}, i != j, iff a_ij or a_ji is stored, */
/* weight |a_ij| + |a_ji| (absent entries count as 0).                       */
/* ------------------------------------------------------------------------ */
static int transpose(const csr_t *A, csr_t *T) {
    int n = A->n, nnz = A->rp[n];
    T->n = n;
    T->rp = calloc((size_t)n + 1, sizeof(int));
    T->ci = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    T->v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!T->rp || !T->ci || !T->v) return OR_ERR_OOM;
    for (int p = 0; p < nnz; ++p) T->rp[A->ci[p] + 1]++;
    for (int i = 0; i < n; ++i) T->rp[i + 1] += T->rp[i];
    int *fill = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!fill) return OR_ERR_OOM;
    memcpy(fill, T->rp, sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int q = fill[A->ci[p]]++;
            T->ci[q] = i;
            T->v[q] = A->v[p];
        }
    free(fill);
    return OR_OK;
}

static int build_graph(const csr_t *A, csr_t *G) {
    csr_t T = {0};
    int st = transpose(A, &T);
    if (st) { csr_free(&T); return st; }
    int n = A->n;
    G->n = n;
    G->rp = calloc((size_t)n + 1, sizeof(int));
    int cap = 2 * A->rp[n] + 1;
    G->ci = malloc(sizeof(int) * (size_t)cap);
    G->v = malloc(sizeof(double) * (size_t)cap);
    if (!G->rp || !G->ci || !G->v) { csr_free(&T); return OR_ERR_OOM; }
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
        int p = A->rp[i], pe = A->rp[i + 1], q = T.rp[i], qe = T.rp[i + 1];
        while (p < pe || q < qe) {
            int cp = p < pe ? A->ci[p] : n, cq = q < qe ? T.ci[q] : n;
            int j = cp < cq ? cp : cq;
            double aij = 0.0, aji = 0.0;
            if (cp == j) { aij = A->v[p]; ++p; }
            if (cq == j) { aji = T.v[q]; ++q; }
            if (j == i) continue;
            G->ci[cnt] = j;
            G->v[cnt] = fabs(aij) + fabs(aji);
            ++cnt;
        }
        G->rp[i + 1] = cnt;
    }
    csr_free(&T);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One handshake matching pass on a symmetric weighted graph (nv vertices):  */
/* in every round each unmatched vertex points at its best unmatched         */
/* neighbour; mutual pointers are matched; rounds repeat until no edge joins */
/* two unmatched vertices (the matching is maximal).                         */
/* ------------------------------------------------------------------------ */
int or_match_once(int nv, const int *rp, const int *ci, const double *w, int qbits,
                  uint64_t seed, int *mate, int *rounds_out) {
    int *cand = malloc(sizeof(int) * (size_t)(nv > 0 ? nv : 1));
    if (!cand) return OR_ERR_OOM;
    for (int v = 0; v < nv; ++v) mate[v] = -1;
    int rounds = 0;
    for (;;) {
        int any = 0;
        for (int v = 0; v < nv; ++v) {
            cand[v] = -1;
            if (mate[v] >= 0) continue;
            ekey best = {0, 0, 0, 0};
            for (int p = rp[v]; p < rp[v + 1]; ++p) {
                int u = ci[p];
                if (u == v || mate[u] >= 0) continue;
                ekey k = make_key(w[p], v, u, qbits, seed);
                if (cand[v] < 0 || key_greater(&k, &best)) { best = k; cand[v] = u; }
            }
            if (cand[v] >= 0) any = 1;
        }
        if (!any) break;
        ++rounds;
        for (int v = 0; v < nv; ++v) {
            int u = cand[v];
            if (u >= 0 && cand[u] == v) mate[v] = u;
        }
    }
    free(cand);
    if (rounds_out) *rounds_out = rounds;
    return OR_OK;
}

/* sort helpers: (row, col, seq) triples, seq keeps the visiting order */
typedef struct { int r, c; long s; double v; } trip;

static int trip_cmp(const void *a, const void *b) {
    const trip *x = a, *y = b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return (x->s > y->s) - (x->s < y->s);
}

/* Sum runs of equal (r, c) in visiting order into a CSR with n rows. */
static int trips_to_csr(trip *t, long nt, int n, csr_t *M) {
    qsort(t, (size_t)nt, sizeof(trip), trip_cmp);
    M->n = n;
    M->rp = calloc((size_t)n + 1, sizeof(int));
    M->ci = malloc(sizeof(int) * (size_t)(nt > 0 ? nt : 1));
    M->v = malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    if (!M->rp || !M->ci || !M->v) return OR_ERR_OOM;
    long k = 0;
    int cnt = 0;
    while (k < nt) {
        long e = k;
        double s = t[k].v;
        while (e + 1 < nt && t[e + 1].r == t[k].r && t[e + 1].c == t[k].c) { ++e; s = s + t[e].v; }
        M->ci[cnt] = t[k].c;
        M->v[cnt] = s;
        M->rp[t[k].r + 1]++;
        ++cnt;
        k = e + 1;
    }
    for (int i = 0; i < n; ++i) M->rp[i + 1] += M->rp[i];
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Multi-pass aggregation.  After each pass aggregates are renumbered by     */
/* their smallest fine index; the next pass works on the aggregate graph    */
/* whose weight w_IJ (I < J) sums the fine graph weights of entries (k, l)   */
/* with agg k = I, agg l = J in CSR order, mirrored to w_JI.                 */
/* ------------------------------------------------------------------------ */
static int aggregate(or_solver *S) {
    int n = S->A.n;
    const csr_t *G0 = &S->G;
    S->agg = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!S->agg) return OR_ERR_OOM;
    for (int k = 0; k < n; ++k) S->agg[k] = k;
    int nv = n;
    long target = (long)floor((double)n / S->o.cf);
    csr_t Gc = {0};
    /* current graph: pass 1 uses G0 itself */
    const int *grp = G0->rp, *gci = G0->ci;
    const double *gw = G0->v;
    S->passes = 0;
    S->rounds = 0;
    int *mate = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *nid = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    trip *t = malloc(sizeof(trip) * (size_t)(G0->rp[n] > 0 ? G0->rp[n] : 1));
    if (!mate || !nid || !t) return OR_ERR_OOM;
    while (nv > target && S->passes < S->o.max_passes) {
        int rounds = 0;
        int st = or_match_once(nv, grp, gci, gw, S->o.qbits, S->o.seed, mate, &rounds);
        if (st) return st;
        int pairs = 0, cnt = 0;
        for (int v = 0; v < nv; ++v) {
            if (mate[v] < 0 || v < mate[v]) { nid[v] = cnt++; if (mate[v] >= 0) ++pairs; }
            else nid[v] = nid[mate[v]];
        }
        if (pairs == 0) break;
        S->passes++;
        S->rounds += rounds;
        for (int k = 0; k < n; ++k) S->agg[k] = nid[S->agg[k]];
        nv = cnt;
        /* aggregate graph for the next pass */
        long nt = 0;
        for (int k = 0; k < n; ++k)
            for (int p = G0->rp[k]; p < G0->rp[k + 1]; ++p) {
                int I = S->agg[k], J = S->agg[G0->ci[p]];
                if (I < J) { t[nt].r = I; t[nt].c = J; t[nt].s = nt; t[nt].v = G0->v[p]; ++nt; }
            }
        csr_t U = {0};
        st = trips_to_csr(t, nt, nv, &U);
        if (st) return st;
        /* mirror: w_JI = w_IJ */
        long nu = U.rp[nv];
        trip *m = malloc(sizeof(trip) * (size_t)(2 * nu > 0 ? 2 * nu : 1));
        if (!m) return OR_ERR_OOM;
        long q = 0;
        for (int I = 0; I < nv; ++I)
            for (int p = U.rp[I]; p < U.rp[I + 1]; ++p) {
                m[q].r = I; m[q].c = U.ci[p]; m[q].v = U.v[p]; m[q].s = q; ++q;
                m[q].r = U.ci[p]; m[q].c = I; m[q].v = U.v[p]; m[q].s = q; ++q;
            }
        csr_free(&U);
        csr_free(&Gc);
        st = trips_to_csr(m, q, nv, &Gc);
        free(m);
        if (st) return st;
        grp = Gc.rp; gci = Gc.ci; gw = Gc.v;
    }
    free(t); free(mate); free(nid);
    csr_free(&Gc);
    S->nc = nv;
    return OR_OK;
}

static int members(or_solver *S) {
    int n = S->A.n, nc = S->nc;
    S->aptr = calloc((size_t)nc + 1, sizeof(int));
    S->amem = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!S->aptr || !S->amem) return OR_ERR_OOM;
    for (int k = 0; k < n; ++k) S->aptr[S->agg[k] + 1]++;
    for (int I = 0; I < nc; ++I) S->aptr[I + 1] += S->aptr[I];
    int *fill = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    if (!fill) return OR_ERR_OOM;
    memcpy(fill, S->aptr, sizeof(int) * (size_t)nc);
    for (int k = 0; k < n; ++k) S->amem[fill[S->agg[k]]++] = k;
    free(fill);
    return OR_OK;
}

/* (A_c)_IJ = sum over k in G_I, l in G_J of a_kl, visited in A's CSR order */
static int galerkin(or_solver *S) {
    const csr_t *A = &S->A;
    long nnz = A->rp[A->n];
    trip *t = malloc(sizeof(trip) * (size_t)(nnz > 0 ? nnz : 1));
    if (!t) return OR_ERR_OOM;
    long nt = 0;
    for (int k = 0; k < A->n; ++k)
        for (int p = A->rp[k]; p < A->rp[k + 1]; ++p) {
            t[nt].r = S->agg[k]; t[nt].c = S->agg[A->ci[p]]; t[nt].v = A->v[p]; t[nt].s = nt; ++nt;
        }
    int st = trips_to_csr(t, nt, S->nc, &S->Ac);
    free(t);
    return st;
}


/* ------------------------------------------------------------------------ */
/* Nested-dissection numbering of the coarse unknowns (the paper reorders by  */
/* nested dissection so that incomplete factors can be computed and applied  */
/* in parallel, Section 3 comments; Table T:norm factors the coarse matrix   */
/* under that ordering).  Graph: i ~ j (i != j) when (A_c)_ij or (A_c)_ji is */
/* stored.  ND(S), S a vertex set:                                           */
/*   |S| <= 64: S ascending.                                                 */
/*   S disconnected: its connected components, ordered by smallest vertex,   */
/*     each numbered by ND.                                                  */
/*   otherwise: BFS from min S; r = smallest vertex at the largest distance; */
/*     d = BFS distance from r within S, L = max d; L < 2: S ascending;       */
/*     m = smallest level with #{d <= m} >= |S|/2, clamped to [1, L-1];       */
/*     ND({d < m}), then ND({d > m}), then {d == m} ascending.               */
/* ------------------------------------------------------------------------ */
#define ND_LEAF 64

static int bfs_in_set(const int *rp, const int *ci, const int *stamp, int tag, int src, int *dist, int *queue) {
    int head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int u = queue[head++];
        for (int p = rp[u]; p < rp[u + 1]; ++p) {
            int v = ci[p];
            if (stamp[v] == tag && dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
        }
    }
    return tail;
}

/* stable partition of seg[0..len) by key[v] in {0,1,2}: returns counts */
static void part3(int *seg, int len, const int *key, int *tmp, int *c0, int *c1) {
    int n0 = 0, n1 = 0, k = 0;
    for (int i = 0; i < len; ++i) if (key[seg[i]] == 0) tmp[k++] = seg[i];
    n0 = k;
    for (int i = 0; i < len; ++i) if (key[seg[i]] == 1) tmp[k++] = seg[i];
    n1 = k - n0;
    for (int i = 0; i < len; ++i) if (key[seg[i]] == 2) tmp[k++] = seg[i];
    memcpy(seg, tmp, sizeof(int) * (size_t)len);
    *c0 = n0; *c1 = n1;
}

/* perm[k] = coarse vertex placed at position k */
static int nd_order(const csr_t *Ac, int *perm) {
    int n = Ac->n;
    csr_t T = {0};
    int st = transpose(Ac, &T);
    if (st) { csr_free(&T); return st; }
    int *rp = malloc(sizeof(int) * ((size_t)n + 1));
    int *ci = malloc(sizeof(int) * (size_t)(2 * Ac->rp[n] + 1));
    int *seq = malloc(sizeof(int) * (size_t)(n + 1)), *tmp = malloc(sizeof(int) * (size_t)(n + 1));
    int *stamp = malloc(sizeof(int) * (size_t)(n + 1)), *dist = malloc(sizeof(int) * (size_t)(n + 1));
    int *queue = malloc(sizeof(int) * (size_t)(n + 1)), *key = malloc(sizeof(int) * (size_t)(n + 1));
    int *cnt = malloc(sizeof(int) * (size_t)(n + 2));
    /* task stack: (kind, start, len); kind 0 = number by ND, 1 = emit */
    int cap = 64, top = 0;
    int *tk = malloc(sizeof(int) * 3 * (size_t)cap);
    if (!rp || !ci || !seq || !tmp || !stamp || !dist || !queue || !key || !cnt || !tk) return OR_ERR_OOM;
    /* symmetric pattern without the diagonal */
    int e = 0;
    rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        int p = Ac->rp[i], pe = Ac->rp[i + 1], q = T.rp[i], qe = T.rp[i + 1];
        while (p < pe || q < qe) {
            int a = p < pe ? Ac->ci[p] : n, b = q < qe ? T.ci[q] : n;
            int j = a < b ? a : b;
            if (a == j) ++p;
            if (b == j) ++q;
            if (j != i) ci[e++] = j;
        }
        rp[i + 1] = e;
    }
    csr_free(&T);
    for (int i = 0; i < n; ++i) { seq[i] = i; stamp[i] = -1; dist[i] = -1; }
    int out = 0, tag = 0;
    tk[0] = 0; tk[1] = 0; tk[2] = n; top = 1;
    while (top > 0) {
        --top;
        int kind = tk[3 * top], s0 = tk[3 * top + 1], len = tk[3 * top + 2];
        int *seg = seq + s0;
        if (len == 0) continue;
        if (kind == 1 || len <= ND_LEAF) {
            for (int i = 0; i < len; ++i) perm[out++] = seg[i];
            continue;
        }
        ++tag;
        for (int i = 0; i < len; ++i) { stamp[seg[i]] = tag; dist[seg[i]] = -1; }
        int reached = bfs_in_set(rp, ci, stamp, tag, seg[0], dist, queue);
        int push[9], np = 0;   /* up to three tasks, pushed in reverse processing order */
        if (reached < len) {
            /* component of min S first, the rest after */
            for (int i = 0; i < len; ++i) key[seg[i]] = dist[seg[i]] >= 0 ? 0 : 1;
            int c0, c1;
            part3(seg, len, key, tmp, &c0, &c1);
            push[np++] = 0; push[np++] = s0 + c0; push[np++] = c1;
            push[np++] = 0; push[np++] = s0; push[np++] = c0;
        } else {
            int far = 0, r = -1;
            for (int i = 0; i < len; ++i) {
                int v = seg[i];
                if (dist[v] > far || (dist[v] == far && (r < 0 || v < r))) { far = dist[v]; r = v; }
            }
            for (int i = 0; i < len; ++i) dist[seg[i]] = -1;
            bfs_in_set(rp, ci, stamp, tag, r, dist, queue);
            int L = 0;
            for (int i = 0; i < len; ++i) if (dist[seg[i]] > L) L = dist[seg[i]];
            if (L < 2) {
                push[np++] = 1; push[np++] = s0; push[np++] = len;
            } else {
                for (int l = 0; l <= L; ++l) cnt[l] = 0;
                for (int i = 0; i < len; ++i) cnt[dist[seg[i]]]++;
                int m = 0, cum = cnt[0];
                while ((double)cum < (double)len / 2.0) { ++m; cum += cnt[m]; }
                if (m < 1) m = 1;
                if (m > L - 1) m = L - 1;
                for (int i = 0; i < len; ++i) {
                    int d = dist[seg[i]];
                    key[seg[i]] = d < m ? 0 : (d > m ? 1 : 2);
                }
                int c0, c1;
                part3(seg, len, key, tmp, &c0, &c1);
                push[np++] = 1; push[np++] = s0 + c0 + c1; push[np++] = len - c0 - c1;
                push[np++] = 0; push[np++] = s0 + c0; push[np++] = c1;
                push[np++] = 0; push[np++] = s0; push[np++] = c0;
            }
        }
        if (top + 3 > cap) { cap *= 2; tk = realloc(tk, sizeof(int) * 3 * (size_t)cap); if (!tk) return OR_ERR_OOM; }
        for (int t = 0; t < np; t += 3) {
            tk[3 * top] = push[t]; tk[3 * top + 1] = push[t + 1]; tk[3 * top + 2] = push[t + 2]; ++top;
        }
    }
    free(rp); free(ci); free(seq); free(tmp); free(stamp); free(dist); free(queue); free(key); free(cnt); free(tk);
    return out == n ? OR_OK : OR_ERR_INVALID;
}

/* renumber aggregates so that A_c's rows follow perm; rebuild P^T and A_c */
static int renumber_coarse(or_solver *S) {
    int nc = S->nc;
    int *perm = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1)), *rank = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    if (!perm || !rank) return OR_ERR_OOM;
    int st = nd_order(&S->Ac, perm);
    if (!st) {
        for (int k = 0; k < nc; ++k) rank[perm[k]] = k;
        for (int k = 0; k < S->A.n; ++k) S->agg[k] = rank[S->agg[k]];
        free(S->aptr); free(S->amem); S->aptr = NULL; S->amem = NULL;
        csr_free(&S->Ac);
        st = members(S);
        if (!st) st = galerkin(S);
    }
    free(perm); free(rank);
    return st;
}

/* ------------------------------------------------------------------------ */
/* The smoother's matrix F.  GMG-ND (the variant list of Section 3.1 and its */
/* comments) reorders the unknowns by nested dissection before ILU(0) so that */
/* the smoother can be built and applied in parallel: F = Q A Q^T, row k of  */
/* F being row fperm[k] of A with columns renumbered and sorted, fperm the   */
/* same dissection rule as the coarse numbering applied to A's graph.        */
/* ------------------------------------------------------------------------ */
static int pair_cmp(const void *a, const void *b) {
    const int *x = a, *y = b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

/* Greedy colouring in natural order: vertex i takes the smallest colour not
   used by a neighbour j < i (i ~ j when a_ij or a_ji is stored); perm lists
   the vertices by colour, ascending within a colour.  On a 2D or 3D grid with
   a 5- or 7-point stencil this is the red-black ordering. */
static int color_order(const csr_t *A, int *perm) {
    int n = A->n;
    csr_t T = {0};
    int st = transpose(A, &T);
    int *color = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *seen = malloc(sizeof(int) * (size_t)(n + 1));
    int *cnt = malloc(sizeof(int) * (size_t)(n + 2));
    if (st || !color || !seen || !cnt) { csr_free(&T); free(color); free(seen); free(cnt); return st ? st : OR_ERR_OOM; }
    for (int c = 0; c <= n; ++c) seen[c] = -1;
    int ncol = 0;
    for (int i = 0; i < n; ++i) {
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) if (A->ci[p] < i) seen[color[A->ci[p]]] = i;
        for (int p = T.rp[i]; p < T.rp[i + 1]; ++p) if (T.ci[p] < i) seen[color[T.ci[p]]] = i;
        int c = 0;
        while (seen[c] == i) ++c;
        color[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    for (int c = 0; c <= ncol; ++c) cnt[c] = 0;
    for (int i = 0; i < n; ++i) cnt[color[i] + 1]++;
    for (int c = 0; c < ncol; ++c) cnt[c + 1] += cnt[c];
    for (int i = 0; i < n; ++i) perm[cnt[color[i]]++] = i;
    csr_free(&T); free(color); free(seen); free(cnt);
    return OR_OK;
}

static int smoother_matrix(or_solver *S) {
    const csr_t *A = &S->A;
    int n = A->n, nnz = A->rp[n];
    S->F.n = n;
    S->F.rp = malloc(sizeof(int) * ((size_t)n + 1));
    S->F.ci = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    S->F.v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    S->fperm = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!S->F.rp || !S->F.ci || !S->F.v || !S->fperm) return OR_ERR_OOM;
    if (S->o.fine_order == 0) {
        for (int k = 0; k < n; ++k) S->fperm[k] = k;
        memcpy(S->F.rp, A->rp, sizeof(int) * ((size_t)n + 1));
        memcpy(S->F.ci, A->ci, sizeof(int) * (size_t)nnz);
        memcpy(S->F.v, A->v, sizeof(double) * (size_t)nnz);
        return OR_OK;
    }
    int st = S->o.fine_order == 1 ? nd_order(A, S->fperm) : color_order(A, S->fperm);
    if (st) return st;
    int *rank = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *pr = malloc(sizeof(int) * 2 * (size_t)(n > 0 ? n : 1));
    if (!rank || !pr) { free(rank); free(pr); return OR_ERR_OOM; }
    for (int k = 0; k < n; ++k) rank[S->fperm[k]] = k;
    S->F.rp[0] = 0;
    for (int k = 0; k < n; ++k) {
        int i = S->fperm[k], len = A->rp[i + 1] - A->rp[i];
        for (int q = 0; q < len; ++q) { pr[2 * q] = rank[A->ci[A->rp[i] + q]]; pr[2 * q + 1] = A->rp[i] + q; }
        qsort(pr, (size_t)len, 2 * sizeof(int), pair_cmp);
        for (int q = 0; q < len; ++q) {
            S->F.ci[S->F.rp[k] + q] = pr[2 * q];
            S->F.v[S->F.rp[k] + q] = A->v[pr[2 * q + 1]];
        }
        S->F.rp[k + 1] = S->F.rp[k] + len;
    }
    free(rank); free(pr);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* ILU(0): incomplete LU restricted to the pattern of F (IKJ form).          */
/* ------------------------------------------------------------------------ */
static int ilu0(or_solver *S) {
    const csr_t *A = &S->F;
    int n = A->n;
    S->ilu = malloc(sizeof(double) * (size_t)(A->rp[n] > 0 ? A->rp[n] : 1));
    S->dpos = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *pos = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!S->ilu || !S->dpos || !pos) return OR_ERR_OOM;
    memcpy(S->ilu, A->v, sizeof(double) * (size_t)A->rp[n]);
    for (int j = 0; j < n; ++j) pos[j] = -1;
    double *a = S->ilu;
    for (int i = 0; i < n; ++i) {
        S->dpos[i] = -1;
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            pos[A->ci[p]] = p;
            if (A->ci[p] == i) S->dpos[i] = p;
        }
        if (S->dpos[i] < 0) { free(pos); return OR_ERR_INVALID; }
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int k = A->ci[p];
            if (k >= i) break;
            a[p] = a[p] / a[S->dpos[k]];
            for (int r = S->dpos[k] + 1; r < A->rp[k + 1]; ++r) {
                int j = A->ci[r];
                if (pos[j] >= 0) a[pos[j]] = a[pos[j]] - a[p] * a[r];
            }
        }
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) pos[A->ci[p]] = -1;
        double d = a[S->dpos[i]];
        if (d == 0.0) { free(pos); return OR_ERR_ZERO_PIVOT; }
        if (!isfinite(d)) { free(pos); return OR_ERR_NONFINITE; }
    }
    free(pos);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* ILUT(tau), Saad's row-wise form without a fill cap and without pivoting:  */
/* an entry of row i is dropped when its magnitude is below tau times the    */
/* 2-norm of the original row i; for the L part the magnitude is taken       */
/* before the division by the pivot (as MATLAB's ilu tests L entries), so    */
/* both parts compare quantities of row i's scale.  The diagonal is kept.    */
/* ------------------------------------------------------------------------ */
typedef struct { int *a; int n; } iheap;

static void hpush(iheap *h, int x) {
    int i = h->n++;
    h->a[i] = x;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h->a[p] <= h->a[i]) break;
        int t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
}

static int hpop(iheap *h) {
    int top = h->a[0];
    h->a[0] = h->a[--h->n];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h->a[l] < h->a[m]) m = l;
        if (r < h->n && h->a[r] < h->a[m]) m = r;
        if (m == i) break;
        int t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
    return top;
}

static int int_cmp(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static int ilut(const csr_t *M, double tau, csr_t *L, csr_t *U) {
    int n = M->n;
    double *w = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    char *in = calloc((size_t)(n > 0 ? n : 1), 1);
    int *lst = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    iheap hp = { malloc(sizeof(int) * (size_t)(n > 0 ? n : 1)), 0 };
    long lcap = M->rp[n] + 16, ucap = M->rp[n] + 16;
    L->n = n; U->n = n;
    L->rp = calloc((size_t)n + 1, sizeof(int));
    U->rp = calloc((size_t)n + 1, sizeof(int));
    L->ci = malloc(sizeof(int) * (size_t)lcap); L->v = malloc(sizeof(double) * (size_t)lcap);
    U->ci = malloc(sizeof(int) * (size_t)ucap); U->v = malloc(sizeof(double) * (size_t)ucap);
    if (!w || !in || !lst || !hp.a || !L->rp || !U->rp || !L->ci || !L->v || !U->ci || !U->v)
        return OR_ERR_OOM;
    long nl = 0, nu = 0;
    int st = OR_OK;
    for (int i = 0; i < n && st == OR_OK; ++i) {
        double nrm = 0.0;
        int nz = 0;
        for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) {
            int j = M->ci[p];
            nrm = nrm + M->v[p] * M->v[p];
            w[j] = M->v[p];
            in[j] = 1;
            lst[nz++] = j;
            if (j < i) hpush(&hp, j);
        }
        double ti = tau * sqrt(nrm);
        if (!in[i]) { in[i] = 1; w[i] = 0.0; lst[nz++] = i; }
        while (hp.n > 0) {
            int k = hpop(&hp);
            /* the drop test sees the value before the division by the pivot
               u_kk (stored first in U row k), in the units of row i */
            if (fabs(w[k]) < ti) { w[k] = 0.0; in[k] = 2; continue; }   /* dropped */
            double wk = w[k] / U->v[U->rp[k]];
            w[k] = wk;
            for (int r = U->rp[k] + 1; r < U->rp[k + 1]; ++r) {
                int j = U->ci[r];
                if (!in[j]) { in[j] = 1; w[j] = 0.0; lst[nz++] = j; if (j < i) hpush(&hp, j); }
                else if (in[j] == 2) continue;   /* cannot happen: dropped k < current */
                w[j] = w[j] - wk * U->v[r];
            }
        }
        qsort(lst, (size_t)nz, sizeof(int), int_cmp);
        if (nl + nz > lcap) { lcap = 2 * (nl + nz); L->ci = realloc(L->ci, sizeof(int) * lcap); L->v = realloc(L->v, sizeof(double) * lcap); }
        if (nu + nz > ucap) { ucap = 2 * (nu + nz); U->ci = realloc(U->ci, sizeof(int) * ucap); U->v = realloc(U->v, sizeof(double) * ucap); }
        if (!L->ci || !L->v || !U->ci || !U->v) return OR_ERR_OOM;
        /* diagonal first in U */
        if (w[i] == 0.0) st = OR_ERR_ZERO_PIVOT;
        else if (!isfinite(w[i])) st = OR_ERR_NONFINITE;
        U->ci[nu] = i; U->v[nu] = w[i]; ++nu;
        for (int t = 0; t < nz; ++t) {
            int j = lst[t];
            if (j < i) {
                if (in[j] == 1) { L->ci[nl] = j; L->v[nl] = w[j]; ++nl; }
            } else if (j > i) {
                if (!(fabs(w[j]) < ti)) { U->ci[nu] = j; U->v[nu] = w[j]; ++nu; }
            }
            in[j] = 0; w[j] = 0.0;
        }
        L->rp[i + 1] = (int)nl;
        U->rp[i + 1] = (int)nu;
    }
    free(w); free(in); free(lst); free(hp.a);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Sparse approximate inverse of A_c (coarse_mode 2): a coarse solve that is  */
/* one sparse product, for the parallel inexact coarse solves Section 2 asks */
/* for once the coarse grid is large.  M has A_c's pattern; its column j     */
/* minimises ||A_c m - e_j||_2 over m supported on J = {i : (A_c)_ij stored} */
/* (a static-pattern SPAI).  Only the rows I where some column k in J of A_c */
/* is stored enter, so the problem is the dense least squares                 */
/* min ||A_c(I, J) m - e_j(I)||, solved by Householder QR and back           */
/* substitution; I and J ascending.  The coarse solve is e_c = M r_c.        */
/* ------------------------------------------------------------------------ */
static int spai(or_solver *S) {
    const csr_t *Ac = &S->Ac;
    int nc = S->nc;
    csr_t T = {0}, Mt = {0};
    int st = transpose(Ac, &T);           /* row j of T = column j of A_c */
    if (st) { csr_free(&T); return st; }
    int nt = T.rp[nc];
    Mt.n = nc;
    Mt.rp = malloc(sizeof(int) * ((size_t)nc + 1));
    Mt.ci = malloc(sizeof(int) * (size_t)(nt > 0 ? nt : 1));
    Mt.v = malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    int *pos = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int *I = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    if (!Mt.rp || !Mt.ci || !Mt.v || !pos || !I) { st = OR_ERR_OOM; goto out; }
    memcpy(Mt.rp, T.rp, sizeof(int) * ((size_t)nc + 1));
    memcpy(Mt.ci, T.ci, sizeof(int) * (size_t)nt);
    for (int i = 0; i < nc; ++i) pos[i] = -1;
    for (int j = 0; j < nc && !st; ++j) {
        const int *J = T.ci + T.rp[j];
        int nj = T.rp[j + 1] - T.rp[j], ni = 0;
        for (int c = 0; c < nj; ++c)
            for (int q = T.rp[J[c]]; q < T.rp[J[c] + 1]; ++q)
                if (pos[T.ci[q]] < 0) { pos[T.ci[q]] = 0; I[ni++] = T.ci[q]; }
        qsort(I, (size_t)ni, sizeof(int), int_cmp);
        for (int r = 0; r < ni; ++r) pos[I[r]] = r;
        /* dense A_c(I, J), row-major ni x nj, and e_j(I) */
        double *H = calloc((size_t)ni * nj + 1, sizeof(double)), *b = calloc((size_t)ni + 1, sizeof(double));
        if (!H || !b) { free(H); free(b); st = OR_ERR_OOM; break; }
        for (int c = 0; c < nj; ++c)
            for (int q = T.rp[J[c]]; q < T.rp[J[c] + 1]; ++q) H[(size_t)pos[T.ci[q]] * nj + c] = T.v[q];
        if (pos[j] >= 0) b[pos[j]] = 1.0;
        /* Householder QR: column c is reflected onto -sign(x_c) ||x|| e_c */
        for (int c = 0; c < nj && c < ni; ++c) {
            double nrm = 0.0;
            for (int r = c; r < ni; ++r) nrm = nrm + H[(size_t)r * nj + c] * H[(size_t)r * nj + c];
            nrm = sqrt(nrm);
            if (nrm == 0.0) continue;
            double x0 = H[(size_t)c * nj + c];
            double alpha = x0 >= 0.0 ? -nrm : nrm;
            /* v = x - alpha e_c (stored in place below the diagonal, v_c apart) */
            double vc = x0 - alpha, vtv = vc * vc;
            for (int r = c + 1; r < ni; ++r) vtv = vtv + H[(size_t)r * nj + c] * H[(size_t)r * nj + c];
            for (int k = c + 1; k < nj; ++k) {
                double d = vc * H[(size_t)c * nj + k];
                for (int r = c + 1; r < ni; ++r) d = d + H[(size_t)r * nj + c] * H[(size_t)r * nj + k];
                double f = 2.0 * d / vtv;
                H[(size_t)c * nj + k] = H[(size_t)c * nj + k] - f * vc;
                for (int r = c + 1; r < ni; ++r) H[(size_t)r * nj + k] = H[(size_t)r * nj + k] - f * H[(size_t)r * nj + c];
            }
            double d = vc * b[c];
            for (int r = c + 1; r < ni; ++r) d = d + H[(size_t)r * nj + c] * b[r];
            double f = 2.0 * d / vtv;
            b[c] = b[c] - f * vc;
            for (int r = c + 1; r < ni; ++r) b[r] = b[r] - f * H[(size_t)r * nj + c];
            H[(size_t)c * nj + c] = alpha;
        }
        /* R m = (Q^T e_j)[0..nj) */
        double *m = Mt.v + T.rp[j];
        for (int c = nj - 1; c >= 0; --c) {
            double t = b[c];
            for (int k = c + 1; k < nj; ++k) t = t - H[(size_t)c * nj + k] * m[k];
            double rcc = H[(size_t)c * nj + c];
            if (rcc == 0.0) { st = OR_ERR_ZERO_PIVOT; break; }
            m[c] = t / rcc;
            if (!isfinite(m[c])) { st = OR_ERR_NONFINITE; break; }
        }
        for (int r = 0; r < ni; ++r) pos[I[r]] = -1;
        free(H); free(b);
    }
    if (!st) st = transpose(&Mt, &S->Mc);
out:
    csr_free(&T); csr_free(&Mt); free(pos); free(I);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Setup                                                                      */
/* ------------------------------------------------------------------------ */
void or_default_opts(or_opts *o) {
    o->cf = 4.0;
    o->max_passes = 8;
    o->qbits = 4;
    o->seed = 0x9E3779B97F4A7C15ULL;
    o->ilut_tau = 1e-4;
    o->coarse_mode = 0;
    o->coarse_sweeps = 3;
    o->coarse_order = 1;
    o->fine_order = 0;
}

void or_destroy(or_solver *S) {
    if (!S) return;
    csr_free(&S->A); csr_free(&S->G); csr_free(&S->Ac); csr_free(&S->Lc); csr_free(&S->Uc);
    csr_free(&S->F); free(S->fperm); csr_free(&S->Mc); free(S->mc32);
    free(S->agg); free(S->aptr); free(S->amem); free(S->ilu); free(S->dpos);
    free(S->v32); free(S->ilu32); free(S->lc32); free(S->uc32);
    free(S);
}

/* agg_given: optional aggregate map (values 0..nc-1, every aggregate
   non-empty, ids ordered by smallest member); NULL runs the matching. */
int or_setup(int n, const int *rp, const int *ci, const double *v, const or_opts *opts,
             const int *agg_given, or_solver **out) {
    *out = NULL;
    if (n < 0 || !rp) return OR_ERR_INVALID;
    or_solver *S = calloc(1, sizeof(or_solver));
    if (!S) return OR_ERR_OOM;
    S->o = *opts;
    if (S->o.qbits < 0 || S->o.qbits > 52 || !(S->o.cf >= 1.0) || S->o.coarse_order < 0 || S->o.coarse_order > 1 ||
        S->o.fine_order < 0 || S->o.fine_order > 2 || S->o.coarse_mode < 0 || S->o.coarse_mode > 2) {
        or_destroy(S);
        return OR_ERR_INVALID;
    }
    if (rp[0] != 0) { or_destroy(S); return OR_ERR_INVALID; }
    for (int i = 0; i < n; ++i) if (rp[i + 1] < rp[i]) { or_destroy(S); return OR_ERR_INVALID; }
    int nnz = rp[n];
    S->A.n = n;
    S->A.rp = malloc(sizeof(int) * ((size_t)n + 1));
    S->A.ci = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    S->A.v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!S->A.rp || !S->A.ci || !S->A.v) { or_destroy(S); return OR_ERR_OOM; }
    memcpy(S->A.rp, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(S->A.ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(S->A.v, v, sizeof(double) * (size_t)nnz);
    for (int p = 0; p < nnz; ++p) if (!isfinite(v[p])) { or_destroy(S); return OR_ERR_NONFINITE; }
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] < 0 || ci[p] >= n || (p > rp[i] && ci[p] <= ci[p - 1])) { or_destroy(S); return OR_ERR_INVALID; }
    int st = build_graph(&S->A, &S->G);
    if (!st) {
        if (agg_given) {
            S->agg = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
            if (!S->agg) st = OR_ERR_OOM;
            else {
                int mx = -1;
                for (int k = 0; k < n; ++k) { S->agg[k] = agg_given[k]; if (agg_given[k] > mx) mx = agg_given[k]; }
                S->nc = mx + 1;
            }
        } else {
            st = aggregate(S);
        }
    }
    if (!st) st = members(S);
    if (!st) st = galerkin(S);
    if (!st && !agg_given && S->o.coarse_order == 1) st = renumber_coarse(S);
    if (!st) st = smoother_matrix(S);
    if (!st) st = ilu0(S);
    if (!st) st = ilut(&S->Ac, S->o.ilut_tau, &S->Lc, &S->Uc);
    if (!st && S->o.coarse_mode == 2) st = spai(S);
    if (!st) {
        S->v32 = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
        S->ilu32 = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
        int nl = S->Lc.rp[S->nc], nu = S->Uc.rp[S->nc];
        S->lc32 = malloc(sizeof(float) * (size_t)(nl > 0 ? nl : 1));
        S->uc32 = malloc(sizeof(float) * (size_t)(nu > 0 ? nu : 1));
        int nm = S->o.coarse_mode == 2 ? S->Mc.rp[S->nc] : 0;
        S->mc32 = malloc(sizeof(float) * (size_t)(nm > 0 ? nm : 1));
        if (!S->v32 || !S->ilu32 || !S->lc32 || !S->uc32 || !S->mc32) st = OR_ERR_OOM;
        else {
            for (int p = 0; p < nnz; ++p) { S->v32[p] = (float)S->A.v[p]; S->ilu32[p] = (float)S->ilu[p]; }
            for (int p = 0; p < nl; ++p) S->lc32[p] = (float)S->Lc.v[p];
            for (int p = 0; p < nm; ++p) S->mc32[p] = (float)S->Mc.v[p];
            for (int p = 0; p < nu; ++p) S->uc32[p] = (float)S->Uc.v[p];
        }
    }
    if (st) { or_destroy(S); return st; }
    *out = S;
    return OR_OK;
}

/* sizes: n, nc, nnz(A), nnz(Ac), nnz(Lc), nnz(Uc), passes, rounds, nnz(G) */
void or_sizes(const or_solver *S, long *out) {
    out[0] = S->A.n; out[1] = S->nc; out[2] = S->A.rp[S->A.n]; out[3] = S->Ac.rp[S->nc];
    out[4] = S->Lc.rp[S->nc]; out[5] = S->Uc.rp[S->nc]; out[6] = S->passes; out[7] = S->rounds;
    out[8] = S->G.rp[S->A.n];
}

void or_get_agg(const or_solver *S, int *agg) { memcpy(agg, S->agg, sizeof(int) * (size_t)S->A.n); }
void or_get_members(const or_solver *S, int *aptr, int *amem) {
    memcpy(aptr, S->aptr, sizeof(int) * ((size_t)S->nc + 1));
    memcpy(amem, S->amem, sizeof(int) * (size_t)S->A.n);
}
static void get_csr(const csr_t *M, int *rp, int *ci, double *v) {
    memcpy(rp, M->rp, sizeof(int) * ((size_t)M->n + 1));
    memcpy(ci, M->ci, sizeof(int) * (size_t)M->rp[M->n]);
    memcpy(v, M->v, sizeof(double) * (size_t)M->rp[M->n]);
}
void or_get_graph(const or_solver *S, int *rp, int *ci, double *v) { get_csr(&S->G, rp, ci, v); }
void or_get_coarse(const or_solver *S, int *rp, int *ci, double *v) { get_csr(&S->Ac, rp, ci, v); }
void or_get_ilut(const or_solver *S, int *lrp, int *lci, double *lv, int *urp, int *uci, double *uv) {
    get_csr(&S->Lc, lrp, lci, lv);
    get_csr(&S->Uc, urp, uci, uv);
}
void or_get_ilu0(const or_solver *S, double *vals) {
    memcpy(vals, S->ilu, sizeof(double) * (size_t)S->A.rp[S->A.n]);
}
/* the sparse approximate inverse of A_c (coarse_mode 2; A_c's pattern) */
void or_get_spai(const or_solver *S, int *rp, int *ci, double *v) {
    if (!S->Mc.rp) return;   /* no inverse unless coarse_mode 2 */
    get_csr(&S->Mc, rp, ci, v);
}
/* the smoother's numbering (position -> fine unknown) and matrix F */
void or_get_fine(const or_solver *S, int *perm, int *rp, int *ci, double *v) {
    memcpy(perm, S->fperm, sizeof(int) * (size_t)S->A.n);
    get_csr(&S->F, rp, ci, v);
}

/* ------------------------------------------------------------------------ */
/* Preconditioner application (the one-coarse-solve form of SOLVE B~q = z):  */
/*   t = U0^{-1} L0^{-1} z,  r = z - A t,  r_c = P^T r,                      */
/*   e_c = U~^{-1} L~^{-1} r_c,  q = t + P e_c.                              */
/* By linearity this equals Algorithm 1's t + f - q with f = M~^{-1} z and   */
/* the second coarse solve applied to A t.                                   */
/* ------------------------------------------------------------------------ */
#define DEFINE_APPLY(T, SUF, AV, ILU, LCV, UCV, MCV)                                            \
/* t = S^{-1} z, S = Q^T L0 U0 Q: u = Q z, y = L0^{-1} u, u = U0^{-1} y, t = Q^T u */  \
static void fine_smooth_##SUF(const or_solver *S, const T *z, T *y, T *t, T *u) {         \
    const csr_t *F = &S->F;                                                                \
    int n = F->n;                                                                          \
    for (int k = 0; k < n; ++k) u[k] = z[S->fperm[k]];                                     \
    for (int i = 0; i < n; ++i) {                                                          \
        T s = u[i];                                                                        \
        for (int p = F->rp[i]; p < S->dpos[i]; ++p) s = s - (T)(ILU)[p] * y[F->ci[p]];     \
        y[i] = s;                                                                          \
    }                                                                                      \
    for (int i = n - 1; i >= 0; --i) {                                                     \
        T s = y[i];                                                                        \
        for (int p = S->dpos[i] + 1; p < F->rp[i + 1]; ++p) s = s - (T)(ILU)[p] * u[F->ci[p]]; \
        u[i] = s / (T)(ILU)[S->dpos[i]];                                                   \
    }                                                                                      \
    for (int k = 0; k < n; ++k) t[S->fperm[k]] = u[k];                                     \
}                                                                                          \
static void coarse_solve_##SUF(const or_solver *S, const T *rc, T *yc, T *ec, T *tmp) {   \
    int nc = S->nc;                                                                        \
    const csr_t *L = &S->Lc, *U = &S->Uc;                                                  \
    if (S->o.coarse_mode == 0) {                                                           \
        for (int i = 0; i < nc; ++i) {                                                     \
            T s = rc[i];                                                                   \
            for (int p = L->rp[i]; p < L->rp[i + 1]; ++p) s = s - (T)(LCV)[p] * yc[L->ci[p]]; \
            yc[i] = s;                                                                     \
        }                                                                                  \
        for (int i = nc - 1; i >= 0; --i) {                                                \
            T s = yc[i];                                                                   \
            for (int p = U->rp[i] + 1; p < U->rp[i + 1]; ++p) s = s - (T)(UCV)[p] * ec[U->ci[p]]; \
            ec[i] = s / (T)(UCV)[U->rp[i]];                                                \
        }                                                                                  \
        return;                                                                            \
    }                                                                                      \
    if (S->o.coarse_mode == 2) {                                                           \
        const csr_t *M = &S->Mc;                                                           \
        for (int i = 0; i < nc; ++i) {                                                     \
            T s = (T)0;                                                                    \
            for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) s = s + (T)(MCV)[p] * rc[M->ci[p]]; \
            ec[i] = s;                                                                     \
        }                                                                                  \
        return;                                                                            \
    }                                                                                      \
    /* Jacobi sweeps on each factor: y <- D^{-1} (b - (F - D) y), y0 = D^{-1} b */        \
    for (int i = 0; i < nc; ++i) yc[i] = rc[i];                                            \
    for (int s = 0; s < S->o.coarse_sweeps; ++s) {                                         \
        for (int i = 0; i < nc; ++i) {                                                     \
            T a = rc[i];                                                                   \
            for (int p = L->rp[i]; p < L->rp[i + 1]; ++p) a = a - (T)(LCV)[p] * yc[L->ci[p]]; \
            tmp[i] = a;                                                                    \
        }                                                                                  \
        for (int i = 0; i < nc; ++i) yc[i] = tmp[i];                                       \
    }                                                                                      \
    for (int i = 0; i < nc; ++i) ec[i] = yc[i] / (T)(UCV)[U->rp[i]];                       \
    for (int s = 0; s < S->o.coarse_sweeps; ++s) {                                         \
        for (int i = 0; i < nc; ++i) {                                                     \
            T a = yc[i];                                                                   \
            for (int p = U->rp[i] + 1; p < U->rp[i + 1]; ++p) a = a - (T)(UCV)[p] * ec[U->ci[p]]; \
            tmp[i] = a / (T)(UCV)[U->rp[i]];                                               \
        }                                                                                  \
        for (int i = 0; i < nc; ++i) ec[i] = tmp[i];                                       \
    }                                                                                      \
}                                                                                          \
static void apply_##SUF(const or_solver *S, const T *z, T *q, T *w) {                      \
    const csr_t *A = &S->A;                                                                \
    int n = A->n, nc = S->nc;                                                              \
    T *y = w, *t = w + n, *u = w + 2 * n, *rc = w + 3 * n, *yc = rc + nc, *ec = yc + nc;   \
    T *tmp = ec + nc;                                                                      \
    fine_smooth_##SUF(S, z, y, t, u);                                                      \
    for (int I = 0; I < nc; ++I) rc[I] = (T)0;                                             \
    for (int I = 0; I < nc; ++I)                                                           \
        for (int m = S->aptr[I]; m < S->aptr[I + 1]; ++m) {                                \
            int k = S->amem[m];                                                            \
            T r = z[k];                                                                    \
            for (int p = A->rp[k]; p < A->rp[k + 1]; ++p) r = r - (T)(AV)[p] * t[A->ci[p]]; \
            rc[I] = rc[I] + r;                                                             \
        }                                                                                  \
    coarse_solve_##SUF(S, rc, yc, ec, tmp);                                                \
    for (int k = 0; k < n; ++k) q[k] = t[k] + ec[S->agg[k]];                               \
}

DEFINE_APPLY(double, f64, S->A.v, S->ilu, S->Lc.v, S->Uc.v, S->Mc.v)
DEFINE_APPLY(float, f32, S->v32, S->ilu32, S->lc32, S->uc32, S->mc32)

/* workspace doubles needed by or_precond_apply */
long or_work_size(const or_solver *S) { return 3L * S->A.n + 4L * S->nc + 8; }

/* precision 0: FP64; 1: FP32 (z rounded to nearest float on entry, every
   operation in float on float copies of A and the factors, q widened on exit) */
void or_precond_apply(const or_solver *S, int precision, const double *z, double *q) {
    int n = S->A.n;
    long ws = or_work_size(S);
    if (precision == 0) {
        double *w = malloc(sizeof(double) * (size_t)ws);
        apply_f64(S, z, q, w);
        free(w);
    } else {
        float *w = malloc(sizeof(float) * (size_t)ws);
        float *z32 = malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
        float *q32 = malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
        for (int i = 0; i < n; ++i) z32[i] = (float)z[i];
        apply_f32(S, z32, q32, w);
        for (int i = 0; i < n; ++i) q[i] = (double)q32[i];
        free(w); free(z32); free(q32);
    }
}

static void spmv(const csr_t *A, const double *x, double *y) {
    for (int i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) s = s + A->v[p] * x[A->ci[p]];
        y[i] = s;
    }
}

static void spmv_t(const csr_t *A, const double *x, double *y) {
    for (int j = 0; j < A->n; ++j) y[j] = 0.0;
    for (int i = 0; i < A->n; ++i)
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p) y[A->ci[p]] = y[A->ci[p]] + A->v[p] * x[i];
}

/* Algorithm 1's literal two-coarse-solve form: t = S^{-1} z, f = M~^{-1} z,
   g = M~^{-1}(A t), q = t + f - g.  Kept for the identity test only. */
void or_precond_apply_twosolve(const or_solver *S, const double *z, double *q) {
    int n = S->A.n, nc = S->nc;
    double *y = malloc(sizeof(double) * (size_t)n), *t = malloc(sizeof(double) * (size_t)n);
    double *at = malloc(sizeof(double) * (size_t)n);
    double *hc = malloc(sizeof(double) * (size_t)nc * 4 + 8);
    double *yc = hc + nc, *fc = yc + nc, *tmp = fc + nc;
    double *gc = malloc(sizeof(double) * (size_t)nc + 8);
    fine_smooth_f64(S, z, y, t, at);
    for (int I = 0; I < nc; ++I) hc[I] = 0.0;
    for (int k = 0; k < n; ++k) hc[S->agg[k]] += z[k];
    coarse_solve_f64(S, hc, yc, fc, tmp);
    spmv(&S->A, t, at);
    for (int I = 0; I < nc; ++I) hc[I] = 0.0;
    for (int k = 0; k < n; ++k) hc[S->agg[k]] += at[k];
    coarse_solve_f64(S, hc, yc, gc, tmp);
    for (int k = 0; k < n; ++k) q[k] = t[k] + fc[S->agg[k]] - gc[S->agg[k]];
    free(y); free(t); free(at); free(hc); free(gc);
}

/* Transpose of the coarse solve, e = M~^{-T} b (b is overwritten).
   coarse_mode 0: U~^T then L~^T by substitution.  coarse_mode 2: e = M^T b.
   coarse_mode 1: the forward solve is J_U J_L with J_L = sum_{i<=k} (-N_L)^i
   (L~ = I + N_L) and J_U = sum_{i<=k} (-D^{-1} N_U)^i D^{-1} (U~ = D + N_U);
   since D^{-1} (-N_U^T D^{-1})^i = (-D^{-1} N_U^T)^i D^{-1}, its transpose
   J_L^T J_U^T is k Jacobi sweeps on U~^T (diagonal D) followed by k sweeps on
   L~^T, the products with N^T taken column by column from the rows of N. */
static void coarse_solve_adjoint(const or_solver *S, double *b, double *e, double *t1, double *t2) {
    int nc = S->nc;
    const csr_t *L = &S->Lc, *U = &S->Uc;
    if (S->o.coarse_mode == 2) {
        const csr_t *M = &S->Mc;
        for (int j = 0; j < nc; ++j) e[j] = 0.0;
        for (int i = 0; i < nc; ++i)
            for (int p = M->rp[i]; p < M->rp[i + 1]; ++p) e[M->ci[p]] = e[M->ci[p]] + M->v[p] * b[i];
        return;
    }
    if (S->o.coarse_mode == 1) {
        /* J_U^T: t1 <- D^{-1} (b - N_U^T t1), t1 = D^{-1} b first */
        for (int i = 0; i < nc; ++i) t1[i] = b[i] / U->v[U->rp[i]];
        for (int sw = 0; sw < S->o.coarse_sweeps; ++sw) {
            for (int i = 0; i < nc; ++i) t2[i] = b[i];
            for (int j = 0; j < nc; ++j)
                for (int p = U->rp[j] + 1; p < U->rp[j + 1]; ++p) t2[U->ci[p]] = t2[U->ci[p]] - U->v[p] * t1[j];
            for (int i = 0; i < nc; ++i) t1[i] = t2[i] / U->v[U->rp[i]];
        }
        /* J_L^T: e <- t1 - N_L^T e, e = t1 first */
        for (int i = 0; i < nc; ++i) e[i] = t1[i];
        for (int sw = 0; sw < S->o.coarse_sweeps; ++sw) {
            for (int i = 0; i < nc; ++i) t2[i] = t1[i];
            for (int j = 0; j < nc; ++j)
                for (int p = L->rp[j]; p < L->rp[j + 1]; ++p) t2[L->ci[p]] = t2[L->ci[p]] - L->v[p] * e[j];
            for (int i = 0; i < nc; ++i) e[i] = t2[i];
        }
        return;
    }
    /* U~^T e = b: U~^T is lower triangular, column-oriented substitution */
    for (int i = 0; i < nc; ++i) {
        e[i] = b[i] / U->v[U->rp[i]];
        for (int p = U->rp[i] + 1; p < U->rp[i + 1]; ++p) b[U->ci[p]] -= U->v[p] * e[i];
    }
    /* L~^T x = e: unit upper triangular */
    for (int i = nc - 1; i >= 0; --i)
        for (int p = L->rp[i]; p < L->rp[i + 1]; ++p) e[L->ci[p]] -= L->v[p] * e[i];
}

/* Transposed preconditioner.  From Eq. (twogrid),
   B~^{-1} = S^{-1} + M~^{-1} (I - A S^{-1}), hence
   B~^{-T} = M~^{-T} + S^{-T} (I - A^T M~^{-T}) with M~^{-T} = P (M~_c)^{-T} P^T
   (M~_c the coarse solve) and S^{-T} = Q^T (L0 U0)^{-T} Q:
     e_c = M~_c^{-T} P^T z,  f = P e_c,  s = z - A^T f,
     t = L0^{-T} U0^{-T} s,  q = f + t. */
void or_precond_apply_adjoint(const or_solver *S, const double *z, double *q) {
    const csr_t *A = &S->A;
    int n = A->n, nc = S->nc;
    double *b = malloc(sizeof(double) * (size_t)nc + 8), *e = malloc(sizeof(double) * (size_t)nc + 8);
    double *t1 = malloc(sizeof(double) * (size_t)nc + 8), *t2 = malloc(sizeof(double) * (size_t)nc + 8);
    double *f = malloc(sizeof(double) * (size_t)n + 8), *s = malloc(sizeof(double) * (size_t)n + 8);
    double *t = malloc(sizeof(double) * (size_t)n + 8);
    double *u = malloc(sizeof(double) * (size_t)n + 8), *tt = malloc(sizeof(double) * (size_t)n + 8);
    const csr_t *F = &S->F;
    for (int I = 0; I < nc; ++I) b[I] = 0.0;
    for (int k = 0; k < n; ++k) b[S->agg[k]] += z[k];
    coarse_solve_adjoint(S, b, e, t1, t2);
    for (int k = 0; k < n; ++k) f[k] = e[S->agg[k]];
    spmv_t(A, f, s);
    for (int k = 0; k < n; ++k) s[k] = z[k] - s[k];
    /* u = Q s; U0^T w = u (lower, with diagonal), then L0^T tt = w (unit
       upper); t = Q^T tt */
    for (int k = 0; k < n; ++k) u[k] = s[S->fperm[k]];
    for (int i = 0; i < n; ++i) {
        tt[i] = u[i] / S->ilu[S->dpos[i]];
        for (int p = S->dpos[i] + 1; p < F->rp[i + 1]; ++p) u[F->ci[p]] -= S->ilu[p] * tt[i];
    }
    for (int i = n - 1; i >= 0; --i)
        for (int p = F->rp[i]; p < S->dpos[i]; ++p) tt[F->ci[p]] -= S->ilu[p] * tt[i];
    for (int k = 0; k < n; ++k) t[S->fperm[k]] = tt[k];
    for (int k = 0; k < n; ++k) q[k] = f[k] + t[k];
    free(b); free(e); free(t1); free(t2); free(f); free(s); free(t); free(u); free(tt);
}

/* ------------------------------------------------------------------------ */
/* Flexible GMRES(m), right preconditioning, modified Gram-Schmidt, Givens   */
/* rotations (Algorithm 1's accelerator with the preconditioner moved to the */
/* right so that each z_j = B~^{-1} v_j is stored).                          */
/* info: [0] steps, [1] restarts, [2] true relres, [3] estimated relres.     */
/* ------------------------------------------------------------------------ */
static double dot(const double *a, const double *b, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

int or_fgmres(const or_solver *S, int adjoint, int precision, const double *b, double *x,
              double tol, int maxit, int m, int x0_given, double *info, double *zdump,
              double *hist, int hist_len) {
    int n = S->A.n;
    if (m < 1) return OR_ERR_INVALID;
    for (int i = 0; i < n; ++i) if (!isfinite(b[i])) return OR_ERR_NONFINITE;
    if (!x0_given) for (int i = 0; i < n; ++i) x[i] = 0.0;
    double *V = malloc(sizeof(double) * (size_t)n * (m + 1) + 8);
    double *Z = malloc(sizeof(double) * (size_t)n * m + 8);
    double *H = calloc((size_t)(m + 1) * m + 1, sizeof(double));
    double *cs = malloc(sizeof(double) * (m + 1)), *sn = malloc(sizeof(double) * (m + 1));
    double *g = malloc(sizeof(double) * (m + 2)), *y = malloc(sizeof(double) * (m + 1));
    double *r = malloc(sizeof(double) * (size_t)n + 8), *w = malloc(sizeof(double) * (size_t)n + 8);
    if (!V || !Z || !H || !cs || !sn || !g || !y || !r || !w) return OR_ERR_OOM;
    double bnorm = sqrt(dot(b, b, n));
    int total = 0, restarts = 0, st = OR_NOT_CONVERGED;
    double relres = 0.0, est = 0.0;
#define HH(i, j) H[(size_t)(i) * m + (j)]
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        st = OR_OK;
        goto done;
    }
    for (;;) {
        if (adjoint) spmv_t(&S->A, x, r); else spmv(&S->A, x, r);
        for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double beta = sqrt(dot(r, r, n));
        relres = beta / bnorm;
        if (!isfinite(relres)) { st = OR_ERR_NONFINITE; break; }
        if (relres < tol) { st = OR_OK; break; }
        if (total >= maxit) { st = OR_NOT_CONVERGED; break; }
        if (total > 0) ++restarts;
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        int breakdown = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            if (adjoint) or_precond_apply_adjoint(S, vj, zj);
            else or_precond_apply(S, precision, vj, zj);
            if (adjoint) spmv_t(&S->A, zj, w); else spmv(&S->A, zj, w);
            for (int i = 0; i <= j; ++i) {
                double h = dot(w, V + (size_t)i * n, n);
                HH(i, j) = h;
                for (int l = 0; l < n; ++l) w[l] = w[l] - h * V[(size_t)i * n + l];
            }
            double hn = sqrt(dot(w, w, n));
            HH(j + 1, j) = hn;
            if (hn != 0.0) for (int l = 0; l < n; ++l) V[(size_t)(j + 1) * n + l] = w[l] / hn;
            for (int i = 0; i < j; ++i) {
                double a = HH(i, j), c = HH(i + 1, j);
                HH(i, j) = cs[i] * a + sn[i] * c;
                HH(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            double rho = hypot(HH(j, j), HH(j + 1, j));
            if (rho == 0.0) { st = OR_ERR_BREAKDOWN; breakdown = 2; break; }
            cs[j] = HH(j, j) / rho;
            sn[j] = HH(j + 1, j) / rho;
            HH(j, j) = rho;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            k = j + 1;
            est = fabs(g[j + 1]) / bnorm;
            if (hist && total <= hist_len) hist[total - 1] = est;
            if (est < tol || hn == 0.0 || total >= maxit) { if (hn == 0.0) breakdown = 1; break; }
        }
        if (breakdown == 2) break;
        /* y = R^{-1} g, x += Z y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s = s - HH(i, l) * y[l];
            y[i] = s / HH(i, i);
        }
        for (int i = 0; i < k; ++i)
            for (int l = 0; l < n; ++l) x[l] = x[l] + y[i] * Z[(size_t)i * n + l];
        if (zdump) memcpy(zdump, Z, sizeof(double) * (size_t)n * k);
        (void)breakdown;
    }
done:
#undef HH
    if (info) { info[0] = total; info[1] = restarts; info[2] = relres; info[3] = est; }
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y); free(r); free(w);
    return st;
}

/* building blocks exposed for tests */
void or_spmv(const or_solver *S, int transposed, const double *x, double *y) {
    if (transposed) spmv_t(&S->A, x, y); else spmv(&S->A, x, y);
}
