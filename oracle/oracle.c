/*
 * Serial FP64 CPU oracle for the Javelin incomplete-LU hot path
 * (Booth & Bolet, "Javelin: A Scalable Implementation for Sparse Incomplete LU
 * Factorization", arXiv:1812.06160).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * reference that the tests, the smoke check and the bench's CPU-baseline leg use
 * to check the HIP library.  The library never links, loads or calls it, and the
 * two share no code.  Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA
 * contraction, no fast-math: every multiply and every subtract is rounded once,
 * IEEE round-to-nearest-even).
 *
 * Every routine is serial and follows the textual definition it cites.  Indices
 * are 0-based; matrices are CSR with int32 row pointers and columns.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_CSR 2
#define ORC_ERR_NOMEM 3
#define ORC_ERR_ZERO_PIVOT 5
#define ORC_ERR_NONFINITE 6
#define ORC_ERR_NOCONV 7
#define ORC_ERR_BREAKDOWN 8

/* qsort comparators: ints ascending; (key, tag) pairs by key then tag.       */
static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}
typedef struct {
    long key;
    long tag;
} orc_pair;
static int cmp_pair(const void *a, const void *b) {
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->tag > y->tag) - (x->tag < y->tag);
}

/* ------------------------------------------------------------------------ */
/* Canonical CSR.  The method takes A in conventional CSR (Sec. I, Sec. II    */
/* "Sparse matrix-vector multiplication and triangular solve").  Columns must */
/* be sorted and unique; a missing diagonal is inserted as an explicit 0.0 so */
/* that the factor pattern always holds the pivot (no pivoting, Sec. III).    */
/* Returns the canonical nnz, or a negative status.  Arrays are written only  */
/* when cap >= the returned size.                                             */
/* ------------------------------------------------------------------------ */
long orc_canonical(int n, const int *rp, const int *ci, const double *v, long cap,
                   int *rp2, int *ci2, double *v2) {
    if (n <= 0 || !rp || !ci) return -ORC_ERR_ARG;
    if (rp[0] != 0) return -ORC_ERR_CSR;
    long need = 0;
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return -ORC_ERR_CSR;
        int has_diag = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) return -ORC_ERR_CSR;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return -ORC_ERR_CSR;
            if (ci[p] == i) has_diag = 1;
        }
        need += (rp[i + 1] - rp[i]) + (has_diag ? 0 : 1);
    }
    if (cap < need) return need;
    long w = 0;
    rp2[0] = 0;
    for (int i = 0; i < n; ++i) {
        int has_diag = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) if (ci[p] == i) has_diag = 1;
        int placed = has_diag;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            if (!placed && ci[p] > i) { ci2[w] = i; v2[w] = 0.0; ++w; placed = 1; }
            ci2[w] = ci[p];
            v2[w] = v ? v[p] : 0.0;
            ++w;
        }
        if (!placed) { ci2[w] = i; v2[w] = 0.0; ++w; }
        rp2[i + 1] = (int)w;
    }
    return need;
}

/* ------------------------------------------------------------------------ */
/* Symbolic ILU(K) by level of fill (the pattern S of Sec. III, whose         */
/* computation the paper delegates to earlier work; Sec. IV "Incomplete       */
/* levels").  Rule: lev = 0 on pattern(A) (diagonal included); processing    */
/* row i, for each k < i in the row's current set in ascending order with    */
/* lev(i,k) <= K, and each j > k in the final row k:                          */
/*     lev(i,j) = min(lev(i,j), lev(i,k) + lev(k,j) + 1),                     */
/* inserting j when absent; entries with lev > K are never kept.              */
/* The row's set is a sorted singly linked list over column indices.          */
/* Input must be canonical.  Returns nnz(S) (negative status on error);      */
/* outputs are written only when cap >= nnz(S).                               */
/* ------------------------------------------------------------------------ */
long orc_symbolic(int n, const int *rp, const int *ci, int K, long cap,
                  int *srp, int *sci, int *slev) {
    if (n <= 0 || K < 0) return -ORC_ERR_ARG;
    long scap = (long)rp[n] + 16, snnz = 0;
    int *Srp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *Sci = (int *)malloc(sizeof(int) * (size_t)scap);
    int *Slev = (int *)malloc(sizeof(int) * (size_t)scap);
    int *next = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *lev = (int *)malloc(sizeof(int) * (size_t)n);
    int *stamp = (int *)malloc(sizeof(int) * (size_t)n);
    if (!Srp || !Sci || !Slev || !next || !lev || !stamp) {
        free(Srp); free(Sci); free(Slev); free(next); free(lev); free(stamp);
        return -ORC_ERR_NOMEM;
    }
    const int END = n;  /* list terminator (larger than every column) */
    const int HEAD = n; /* next[HEAD] is the first column */
    for (int j = 0; j < n; ++j) stamp[j] = -1;
    Srp[0] = 0;
    for (int i = 0; i < n; ++i) {
        /* initial list: the row of A, all at level 0 */
        int last = HEAD;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int j = ci[p];
            next[last] = j;
            last = j;
            lev[j] = 0;
            stamp[j] = i;
        }
        next[last] = END;
        /* walk k ascending through the (growing) list while k < i */
        int k = next[HEAD];
        while (k != END && k < i) {
            int lk = lev[k];
            if (lk <= K) {
                int prev = k; /* insertion cursor: columns of row k ascend */
                for (long q = Srp[k]; q < Srp[k + 1]; ++q) {
                    int j = Sci[q];
                    if (j <= k) continue;
                    int nl = lk + Slev[q] + 1;
                    if (nl > K) continue;
                    if (stamp[j] == i) {
                        if (nl < lev[j]) lev[j] = nl;
                    } else {
                        while (next[prev] < j) prev = next[prev];
                        next[j] = next[prev];
                        next[prev] = j;
                        lev[j] = nl;
                        stamp[j] = i;
                    }
                    prev = j; /* j is now in the list; later j of row k are larger */
                }
            }
            k = next[k];
        }
        /* emit the row */
        for (int j = next[HEAD]; j != END; j = next[j]) {
            if (snnz >= scap) {
                scap = scap * 2;
                int *a = (int *)realloc(Sci, sizeof(int) * (size_t)scap);
                int *b = (int *)realloc(Slev, sizeof(int) * (size_t)scap);
                if (!a || !b) {
                    free(a ? a : Sci); free(b ? b : Slev); free(Srp); free(next); free(lev); free(stamp);
                    return -ORC_ERR_NOMEM;
                }
                Sci = a; Slev = b;
            }
            Sci[snnz] = j;
            Slev[snnz] = lev[j];
            ++snnz;
        }
        Srp[i + 1] = (int)snnz;
    }
    if (cap >= snnz) {
        memcpy(srp, Srp, sizeof(int) * ((size_t)n + 1));
        memcpy(sci, Sci, sizeof(int) * (size_t)snnz);
        memcpy(slev, Slev, sizeof(int) * (size_t)snnz);
    }
    free(Srp); free(Sci); free(Slev); free(next); free(lev); free(stamp);
    return snnz;
}

/* ------------------------------------------------------------------------ */
/* Level sets (Sec. II "Parallel incomplete LU factorization"; Sec. III).     */
/* A row depends on every earlier row j it is connected to in lower(S)       */
/* (sym = 0) or in lower(S + S^T) (sym = 1).  The level of a row is 0 when it */
/* has no dependency, else one more than the largest level among its         */
/* dependencies (the longest dependency path), which is the level a row gets */
/* when rows without incoming edges are peeled off repeatedly.              */
/* Returns the number of levels.                                              */
/* ------------------------------------------------------------------------ */
int orc_levels(int n, const int *rp, const int *ci, int sym, int *level) {
    int *pend = (int *)calloc((size_t)n, sizeof(int));
    if (!pend) return -ORC_ERR_NOMEM;
    int nlev = 0;
    for (int i = 0; i < n; ++i) {
        int L = pend[i];
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int j = ci[p];
            if (j < i && level[j] + 1 > L) L = level[j] + 1;
        }
        level[i] = L;
        if (L + 1 > nlev) nlev = L + 1;
        if (sym) {
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                int j = ci[p];
                if (j > i && L + 1 > pend[j]) pend[j] = L + 1;
            }
        }
    }
    free(pend);
    return nlev;
}

/* Stable counting sort of rows by key (level): perm lists the rows in order  */
/* of (key, original index); iperm is its inverse; ptr[l] is the first        */
/* position of key l (Sec. III: rows are permuted into the level ordering).   */
void orc_sort_by_key(int n, const int *key, int nkey, int *perm, int *iperm, int *ptr) {
    for (int l = 0; l <= nkey; ++l) ptr[l] = 0;
    for (int i = 0; i < n; ++i) ptr[key[i] + 1]++;
    for (int l = 0; l < nkey; ++l) ptr[l + 1] += ptr[l];
    int *fill = (int *)malloc(sizeof(int) * ((size_t)nkey + 1));
    for (int l = 0; l <= nkey; ++l) fill[l] = ptr[l];
    for (int i = 0; i < n; ++i) {
        int r = fill[key[i]]++;
        perm[r] = i;
        if (iperm) iperm[i] = r;
    }
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Reverse Cuthill-McKee preordering (Sec. VII compares it with the natural  */
/* and nested-dissection orderings without stating the algorithm; this is   */
/* the textbook one).  Graph: the pattern of A + A^T without the diagonal;   */
/* deg(v) = number of distinct neighbours.  Components are taken in order of */
/* their smallest vertex.  Start vertex of a component: pseudo-peripheral    */
/* search (George and Liu) from the vertex of least degree (ties: smaller    */
/* index): build the BFS level structure from r, take x = the vertex of      */
/* least degree (ties: smaller index) in its last level; if the structure    */
/* from x is deeper, r = x and repeat, else keep r.  Cuthill-McKee visit:    */
/* breadth first from the start, each vertex's unvisited neighbours queued   */
/* in order of (degree, index).  The whole visit order is then reversed:     */
/* order[i] is the input vertex that becomes vertex i.                       */
/* ------------------------------------------------------------------------ */
/* Breadth-first level structure of the component of root: queue receives  */
/* the component in visit order; returns the depth (levels - 1), with the    */
/* component size in *size and the queue position of the last level's first */
/* vertex in *last_lo.                                                       */
static int rcm_bfs(const int *ap, const int *aj, int root, int *mark, int stamp, int *queue, int *size,
                   int *last_lo) {
    int head = 0, tail = 0, depth = 0, lo = 0, hi = 1;
    queue[tail++] = root;
    mark[root] = stamp;
    while (head < tail) {
        if (head == hi) {   /* every vertex of the current level is expanded */
            ++depth;
            lo = hi;
            hi = tail;
        }
        int u = queue[head++];
        for (int p = ap[u]; p < ap[u + 1]; ++p) {
            int w = aj[p];
            if (mark[w] != stamp) {
                mark[w] = stamp;
                queue[tail++] = w;
            }
        }
    }
    *size = tail;
    *last_lo = lo;
    return depth;
}

static int rcm_less(const int *deg, int a, int b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); }

int orc_rcm(int n, const int *rp, const int *ci, int *order) {
    int *ap = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    int *deg = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *mark = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *visited = (int *)calloc((size_t)n + 1, sizeof(int));
    int *queue = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *cm = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    orc_pair *kids = (orc_pair *)malloc(sizeof(orc_pair) * ((size_t)n + 1));
    if (!ap || !cnt || !deg || !mark || !visited || !queue || !cm || !kids) return ORC_ERR_NOMEM;
    /* adjacency of A + A^T without the diagonal: both directions of every entry */
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                cnt[i + 1]++;
                cnt[ci[p] + 1]++;
            }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int *aj = (int *)malloc(sizeof(int) * ((size_t)cnt[n] + 1));
    if (!aj) return ORC_ERR_NOMEM;
    for (int i = 0; i < n; ++i) mark[i] = cnt[i];   /* next free place of row i */
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                aj[mark[i]++] = ci[p];
                aj[mark[ci[p]]++] = i;
            }
    /* sort each row and squeeze out repeated neighbours */
    ap[0] = 0;
    for (int i = 0; i < n; ++i) {
        int lo = cnt[i], hi = cnt[i + 1];
        qsort(aj + lo, (size_t)(hi - lo), sizeof(int), cmp_int);
        int len = 0;
        for (int a = lo; a < hi; ++a)
            if (len == 0 || aj[ap[i] + len - 1] != aj[a]) aj[ap[i] + len++] = aj[a];
        ap[i + 1] = ap[i] + len;
        deg[i] = len;
    }
    for (int i = 0; i < n; ++i) mark[i] = 0;
    int stamp = 0, ncm = 0;
    for (int v = 0; v < n; ++v) {
        if (visited[v]) continue;
        /* the vertex of least degree of v's component */
        int size, lo;
        rcm_bfs(ap, aj, v, mark, ++stamp, queue, &size, &lo);
        int r = v;
        for (int a = 0; a < size; ++a)
            if (rcm_less(deg, queue[a], r)) r = queue[a];
        /* pseudo-peripheral search */
        int depth = rcm_bfs(ap, aj, r, mark, ++stamp, queue, &size, &lo);
        for (;;) {
            int x = queue[lo];
            for (int a = lo + 1; a < size; ++a)
                if (rcm_less(deg, queue[a], x)) x = queue[a];
            int sx, lx;
            int dx = rcm_bfs(ap, aj, x, mark, ++stamp, queue, &sx, &lx);
            if (dx <= depth) break;
            r = x;
            depth = dx;
            size = sx;
            lo = lx;
        }
        /* Cuthill-McKee visit from r: each vertex's unvisited neighbours in
           (degree, index) order */
        int head = ncm;
        cm[ncm++] = r;
        visited[r] = 1;
        while (head < ncm) {
            int u = cm[head++];
            int nk = 0;
            for (int p = ap[u]; p < ap[u + 1]; ++p) {
                int w = aj[p];
                if (visited[w]) continue;
                visited[w] = 1;
                kids[nk].key = (long)deg[w] * n + w;   /* (degree, index) order */
                kids[nk].tag = w;
                ++nk;
            }
            qsort(kids, (size_t)nk, sizeof(orc_pair), cmp_pair);
            for (int k = 0; k < nk; ++k) cm[ncm++] = (int)kids[k].tag;
        }
    }
    /* reverse */
    for (int i = 0; i < n; ++i) order[i] = cm[n - 1 - i];
    free(ap);
    free(cnt);
    free(deg);
    free(mark);
    free(visited);
    free(queue);
    free(cm);
    free(kids);
    free(aj);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Symmetric permutation P S P^T of a pattern with an integer tag per entry  */
/* (Sec. III: A is copied into the CSR of L and U in level order).  Row r of */
/* the result is the original row perm[r] with each column j renamed         */
/* iperm[j], sorted ascending (qsort).          src[p] is the index of the */
/* source entry; diag_pos[r] is the position of column r (or -1).            */
/* ------------------------------------------------------------------------ */
void orc_permute(int n, const int *rp, const int *ci, const int *perm, const int *iperm,
                 int *prp, int *pci, long *src, int *diag_pos) {
    prp[0] = 0;
    for (int r = 0; r < n; ++r) {
        int i = perm[r];
        int len = rp[i + 1] - rp[i];
        prp[r + 1] = prp[r] + len;
    }
    int maxlen = 0;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > maxlen) maxlen = rp[i + 1] - rp[i];
    orc_pair *row = (orc_pair *)malloc(sizeof(orc_pair) * ((size_t)maxlen + 1));
    for (int r = 0; r < n; ++r) {
        int i = perm[r];
        int base = prp[r];
        int len = rp[i + 1] - rp[i];
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            row[p - rp[i]].key = iperm[ci[p]];
            row[p - rp[i]].tag = p;
        }
        qsort(row, (size_t)len, sizeof(orc_pair), cmp_pair);
        for (int k = 0; k < len; ++k) {
            pci[base + k] = (int)row[k].key;
            src[base + k] = row[k].tag;
        }
        diag_pos[r] = -1;
        for (int p = base; p < base + len; ++p)
            if (pci[p] == r) diag_pos[r] = p;
    }
    free(row);
}

/* Values of A placed on the pattern S (both canonical and sorted by row):   */
/* entries of S that are also entries of A take A's value, fill takes 0.0.   */
/* amap[s] is the index of the A entry (or -1 for fill).                      */
void orc_values_on_pattern(int n, const int *arp, const int *aci, const double *av,
                           const int *srp, const int *sci, double *sval, long *amap) {
    for (int i = 0; i < n; ++i) {
        int q = arp[i];
        for (int s = srp[i]; s < srp[i + 1]; ++s) {
            while (q < arp[i + 1] && aci[q] < sci[s]) ++q;
            if (q < arp[i + 1] && aci[q] == sci[s]) {
                sval[s] = av ? av[q] : 0.0;
                if (amap) amap[s] = q;
            } else {
                sval[s] = 0.0;
                if (amap) amap[s] = -1;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Schedule of the backward (upper) solve.  ulev[r] = 0 when row r of the    */
/* permuted pattern has no column right of the diagonal, else one more than  */
/* the largest ulev over those columns (rows are visited from the last up).  */
/* Returns the number of upper levels.                                       */
/* ------------------------------------------------------------------------ */
int orc_upper_levels(int n, const int *rp, const int *ci, int *ulev) {
    int nlev = 0;
    for (int r = n - 1; r >= 0; --r) {
        int L = 0;
        for (int p = rp[r]; p < rp[r + 1]; ++p) {
            int c = ci[p];
            if (c > r && ulev[c] + 1 > L) L = ulev[c] + 1;
        }
        ulev[r] = L;
        if (L + 1 > nlev) nlev = L + 1;
    }
    return nlev;
}

/* Drop threshold per permuted row: tau_r = tau * ||A(perm[r], :)||_2, the   */
/* 2-norm of the original row taken in ascending column order (ILU(tau),     */
/* Sec. I; the paper names dropping by value without fixing the rule).       */
void orc_row_tau(int n, const int *arp, const double *av, const int *perm, double tau,
                 double *row_tau) {
    for (int r = 0; r < n; ++r) {
        int i = perm[r];
        double s = 0.0;
        for (int p = arp[i]; p < arp[i + 1]; ++p) {
            double sq = av[p] * av[p];
            s = s + sq;
        }
        row_tau[r] = tau * sqrt(s);
    }
}

/* ------------------------------------------------------------------------ */
/* Numeric up-looking incomplete LU on a fixed pattern (Sec. III, Fig. 1).   */
/* L (unit diagonal, strictly lower) and U overwrite val in place.  For each */
/* row r, each kept column c < r is taken in ascending order:                */
/*    a_rc = a_rc / a_cc; if |a_rc| < tau_r the entry is dropped (0, stat 1);*/
/*    else a_rj = a_rj - a_rc * a_cj for each kept j > c of row c that is    */
/*    also a kept column of row r.                                           */
/* Then U entries of row r right of the diagonal with |a_rj| < tau_r are    */
/* dropped.  Entries whose fill level exceeds k are absent (stat 2, 0.0);    */
/* they neither update nor receive updates.  The diagonal is never dropped.  */
/* Modified ILU (milu != 0; Sec. I and Sec. III name it as an option without */
/* defining it; the textbook rule is taken): whatever row r loses is added to */
/* its diagonal at the moment it is lost, so the row sums of L*U equal those */
/* of A.  An update l*u_cj whose target (r, j) is outside the kept pattern   */
/* (not stored, or absent) is subtracted from a_rr; a dropped multiplier     */
/* gives back its value before the division (a_rr += a_rc); a dropped U      */
/* entry gives back its value (a_rr += a_rj), in ascending column order.     */
/* No pivoting (Sec. III): the first row with a_rr == 0 gives ZERO_PIVOT,    */
/* the first row with any non-finite value gives NONFINITE; the oracle stops */
/* there and reports the row in *bad_row.                                    */
/* ------------------------------------------------------------------------ */
int orc_factor(int n, const int *rp, const int *ci, const int *flev, const int *diag_pos,
               double *val, int k, const double *row_tau, int milu, signed char *stat, int *bad_row) {
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    if (!pos) return ORC_ERR_NOMEM;
    for (int j = 0; j < n; ++j) pos[j] = -1;
    *bad_row = -1;
    for (int p = 0; p < rp[n]; ++p) {
        stat[p] = (flev && flev[p] > k) ? 2 : 0;
        if (stat[p] == 2) val[p] = 0.0;
    }
    int status = ORC_OK;
    for (int r = 0; r < n; ++r) {
        double tr = row_tau ? row_tau[r] : 0.0;
        for (int p = rp[r]; p < rp[r + 1]; ++p) pos[ci[p]] = p;
        int dr = diag_pos[r];
        for (int p = rp[r]; p < rp[r + 1] && ci[p] < r; ++p) {
            if (stat[p] != 0) continue;
            int c = ci[p];
            double before = val[p];
            val[p] = val[p] / val[diag_pos[c]];
            if (fabs(val[p]) < tr) {
                val[p] = 0.0;
                stat[p] = 1;
                if (milu) val[dr] = val[dr] + before;
                continue;
            }
            for (int q = diag_pos[c] + 1; q < rp[c + 1]; ++q) {
                if (stat[q] != 0) continue;
                int t = pos[ci[q]];
                if (t < 0 || stat[t] != 0) {
                    if (milu) {
                        double lost = val[p] * val[q];
                        val[dr] = val[dr] - lost;
                    }
                    continue;
                }
                double prod = val[p] * val[q];
                val[t] = val[t] - prod;
            }
        }
        for (int p = dr + 1; p < rp[r + 1]; ++p) {
            if (stat[p] == 0 && fabs(val[p]) < tr) {
                if (milu) val[dr] = val[dr] + val[p];
                val[p] = 0.0;
                stat[p] = 1;
            }
        }
        for (int p = rp[r]; p < rp[r + 1]; ++p) pos[ci[p]] = -1;
        if (val[diag_pos[r]] == 0.0) { status = ORC_ERR_ZERO_PIVOT; *bad_row = r; break; }
        int nonfinite = 0;
        for (int p = rp[r]; p < rp[r + 1]; ++p) if (!isfinite(val[p])) nonfinite = 1;
        if (nonfinite) { status = ORC_ERR_NONFINITE; *bad_row = r; break; }
    }
    free(pos);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Storage precisions for the factor.  FP32: round to nearest even (C cast). */
/* BF16: the FP32 value rounded to nearest even to 8 significand bits (upper */
/* 16 bits of the FP32 pattern); NaN stays NaN (quiet bit set).              */
/* ------------------------------------------------------------------------ */
void orc_cast_f32(long m, const double *x, float *y) {
    for (long i = 0; i < m; ++i) y[i] = (float)x[i];
}

static uint16_t bf16_from_f32(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

static float f32_from_bf16(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

void orc_cast_bf16(long m, const double *x, uint16_t *y) {
    for (long i = 0; i < m; ++i) y[i] = bf16_from_f32((float)x[i]);
}

/* ------------------------------------------------------------------------ */
/* Preconditioner apply x = M^{-1} b = P^T U^{-1} L^{-1} P b (Sec. II,       */
/* "sparse triangular solve"; Sec. VI).  Forward: y_r = b'_r - sum_{c<r}     */
/* l_rc y_c with the unit diagonal implied; backward: x_r = (y_r -           */
/* sum_{c>r} u_rc x_c) / u_rr.  Each sum accumulates in ascending column     */
/* order.  b and x are row-major [n][ld] in the original ordering (perm !=   */
/* NULL) or in the permuted ordering (perm == NULL); y_out (optional)        */
/* receives the permuted intermediate y, [n][ld].                            */
/* ------------------------------------------------------------------------ */
void orc_apply_f64(int n, const int *rp, const int *ci, const int *diag_pos, const double *val,
                   const int *perm, const double *b, double *x, double *y_out, int nrhs, long ld) {
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    for (int s = 0; s < nrhs; ++s) {
        for (int r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int p = rp[r]; p < diag_pos[r]; ++p) {
                double prod = val[p] * y[ci[p]];
                acc = acc + prod;
            }
            double br = b[(long)(perm ? perm[r] : r) * ld + s];
            y[r] = br - acc;
        }
        for (int r = n - 1; r >= 0; --r) {
            double acc = 0.0;
            for (int p = diag_pos[r] + 1; p < rp[r + 1]; ++p) {
                double prod = val[p] * z[ci[p]];
                acc = acc + prod;
            }
            z[r] = (y[r] - acc) / val[diag_pos[r]];
        }
        for (int r = 0; r < n; ++r) {
            x[(long)(perm ? perm[r] : r) * ld + s] = z[r];
            if (y_out) y_out[(long)r * ld + s] = y[r];
        }
    }
    free(y);
    free(z);
}

/* The same apply with FP32 factor values: b is rounded to FP32, every       */
/* operation is FP32, and x is widened to FP64.  prec 1 = FP32 values        */
/* (float*), prec 2 = BF16 values (uint16_t*, widened exactly to FP32).      */
void orc_apply_lowp(int n, const int *rp, const int *ci, const int *diag_pos, const void *valp,
                    int prec, const int *perm, const double *b, double *x, int nrhs, long ld) {
    const float *v32 = (const float *)valp;
    const uint16_t *v16 = (const uint16_t *)valp;
    float *y = (float *)malloc(sizeof(float) * (size_t)n);
    float *z = (float *)malloc(sizeof(float) * (size_t)n);
    for (int s = 0; s < nrhs; ++s) {
        for (int r = 0; r < n; ++r) {
            float acc = 0.0f;
            for (int p = rp[r]; p < diag_pos[r]; ++p) {
                float a = prec == 1 ? v32[p] : f32_from_bf16(v16[p]);
                float prod = a * y[ci[p]];
                acc = acc + prod;
            }
            float br = (float)b[(long)(perm ? perm[r] : r) * ld + s];
            y[r] = br - acc;
        }
        for (int r = n - 1; r >= 0; --r) {
            float acc = 0.0f;
            for (int p = diag_pos[r] + 1; p < rp[r + 1]; ++p) {
                float a = prec == 1 ? v32[p] : f32_from_bf16(v16[p]);
                float prod = a * z[ci[p]];
                acc = acc + prod;
            }
            float d = prec == 1 ? v32[diag_pos[r]] : f32_from_bf16(v16[diag_pos[r]]);
            z[r] = (y[r] - acc) / d;
        }
        for (int r = 0; r < n; ++r) x[(long)(perm ? perm[r] : r) * ld + s] = (double)z[r];
    }
    free(y);
    free(z);
}

/* Sparse matrix-vector product y = A x (Sec. II), ascending column order,  */
/* x and y row-major [n][ld] with nrhs columns.                              */
void orc_spmv(int n, const int *rp, const int *ci, const double *val, const double *x, double *y,
              int nrhs, long ld) {
    for (int s = 0; s < nrhs; ++s)
        for (int r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int p = rp[r]; p < rp[r + 1]; ++p) {
                double prod = val[p] * x[(long)ci[p] * ld + s];
                acc = acc + prod;
            }
            y[(long)r * ld + s] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Krylov consumers of the preconditioner (Sec. I and II: CG and GMRES rely  */
/* on spmv and stri).  Both work on one right-hand side in whatever ordering */
/* the arrays are given (the tests pass the permuted system B = P A P^T,     */
/* b' = P b, and the factor of B).  prec selects the factor storage used by  */
/* the apply: 0 FP64 (val64), 1 FP32 (vlow as float), 2 BF16 (vlow as        */
/* uint16).  The residual, inner products and updates are FP64.              */
/* ------------------------------------------------------------------------ */
static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double p = a[i] * b[i];
        s = s + p;
    }
    return s;
}

static void precond(int n, const int *lrp, const int *lci, const int *ldp, const double *val64,
                    const void *vlow, int prec, const double *r, double *z) {
    if (prec == 0) orc_apply_f64(n, lrp, lci, ldp, val64, NULL, r, z, NULL, 1, 1);
    else orc_apply_lowp(n, lrp, lci, ldp, vlow, prec, NULL, r, z, 1, 1);
}

/* Preconditioned CG (x0 = 0).  Stops when ||r_k|| / ||b|| <= tol on the    */
/* recurrence, then checks the true residual b - A x; if that misses tol,   */
/* the recurrence restarts from the true residual.  out[0] = iterations,    */
/* out[1] = true relative residual.                                          */
int orc_pcg(int n, const int *arp, const int *aci, const double *aval,
            const int *lrp, const int *lci, const int *ldp, const double *val64, const void *vlow,
            int prec, const double *b, double *x, double tol, int maxit, double *out) {
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double bnorm = sqrt(dot(n, b, b));
    int it = 0, status = ORC_ERR_NOCONV;
    for (int i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    double relres = 1.0;
    if (bnorm == 0.0) { status = ORC_OK; relres = 0.0; goto done; }
    for (;;) {
        precond(n, lrp, lci, ldp, val64, vlow, prec, r, z);
        for (int i = 0; i < n; ++i) p[i] = z[i];
        double rz = dot(n, r, z);
        int converged = 0;
        while (it < maxit) {
            orc_spmv(n, arp, aci, aval, p, q, 1, 1);
            double pq = dot(n, p, q);
            if (pq == 0.0) { status = ORC_ERR_BREAKDOWN; goto done; }
            double alpha = rz / pq;
            for (int i = 0; i < n; ++i) {
                double t = alpha * p[i];
                x[i] = x[i] + t;
                double u = alpha * q[i];
                r[i] = r[i] - u;
            }
            ++it;
            if (sqrt(dot(n, r, r)) / bnorm <= tol) { converged = 1; break; }
            precond(n, lrp, lci, ldp, val64, vlow, prec, r, z);
            double rz1 = dot(n, r, z);
            double beta = rz1 / rz;
            rz = rz1;
            for (int i = 0; i < n; ++i) {
                double t = beta * p[i];
                p[i] = z[i] + t;
            }
        }
        /* true residual */
        orc_spmv(n, arp, aci, aval, x, q, 1, 1);
        for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
        relres = sqrt(dot(n, r, r)) / bnorm;
        if (relres <= tol) { status = ORC_OK; break; }
        if (!converged || it >= maxit) { status = ORC_ERR_NOCONV; break; }
    }
done:
    out[0] = it;
    out[1] = relres;
    free(r); free(z); free(p); free(q);
    return status;
}

/* Right-preconditioned flexible GMRES(m) with modified Gram-Schmidt and     */
/* Givens rotations (x0 = 0).  A cycle ends when |g_{j+1}| / ||b|| <= tol,   */
/* at happy breakdown, or after m steps; the true residual decides whether  */
/* to restart.  out[0] = iterations (inner steps), out[1] = true relres.    */
int orc_fgmres(int n, const int *arp, const int *aci, const double *aval,
               const int *lrp, const int *lci, const int *ldp, const double *val64, const void *vlow,
               int prec, const double *b, double *x, double tol, int m, int maxcycles, double *out) {
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(m + 1));
    double *Z = (double *)malloc(sizeof(double) * (size_t)n * (size_t)m);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *yv = (double *)malloc(sizeof(double) * (size_t)m);
    double bnorm = sqrt(dot(n, b, b));
    int it = 0, status = ORC_ERR_NOCONV;
    double relres = 1.0;
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    if (bnorm == 0.0) { status = ORC_OK; relres = 0.0; goto done; }
    for (int cycle = 0; cycle < maxcycles; ++cycle) {
        orc_spmv(n, arp, aci, aval, x, w, 1, 1);
        for (int i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dot(n, w, w));
        relres = beta / bnorm;
        if (relres <= tol) { status = ORC_OK; break; }
        for (int i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int jend = -1;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            precond(n, lrp, lci, ldp, val64, vlow, prec, vj, zj);
            orc_spmv(n, arp, aci, aval, zj, w, 1, 1);
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * n;
                double h = dot(n, w, vi);
                H[(size_t)i * m + j] = h;
                for (int t = 0; t < n; ++t) {
                    double u = h * vi[t];
                    w[t] = w[t] - u;
                }
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn != 0.0) {
                double *vn = V + (size_t)(j + 1) * n;
                for (int t = 0; t < n; ++t) vn[t] = w[t] / hn;
            }
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                double t1 = cs[i] * a, t2 = sn[i] * c;
                double t3 = cs[i] * c, t4 = sn[i] * a;
                H[(size_t)i * m + j] = t1 + t2;
                H[(size_t)(i + 1) * m + j] = t3 - t4;
            }
            double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            double aa = a * a, cc = c * c;
            double den = sqrt(aa + cc);
            cs[j] = a / den;
            sn[j] = c / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -(sn[j] * g[j]);
            g[j] = cs[j] * g[j];
            ++it;
            jend = j;
            if (fabs(g[j + 1]) / bnorm <= tol || hn == 0.0) break;
        }
        for (int i = jend; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t <= jend; ++t) {
                double u = H[(size_t)i * m + t] * yv[t];
                s = s - u;
            }
            yv[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i <= jend; ++i) {
            double *zi = Z + (size_t)i * n;
            for (int t = 0; t < n; ++t) {
                double u = yv[i] * zi[t];
                x[t] = x[t] + u;
            }
        }
    }
    if (status != ORC_OK) {
        orc_spmv(n, arp, aci, aval, x, w, 1, 1);
        for (int i = 0; i < n; ++i) w[i] = b[i] - w[i];
        relres = sqrt(dot(n, w, w)) / bnorm;
        if (relres <= tol) status = ORC_OK;
    }
done:
    out[0] = it;
    out[1] = relres;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(yv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the apply x = P^T U^{-1} L^{-1} P b for a loss with gradient  */
/* gx = dl/dx (original ordering, [n][ld]).  With z = P x and y = L^{-1} P b */
/* (both permuted):                                                          */
/*   w   = U^{-T} P gx         (transposed upper solve, column-push form)    */
/*   b'  = L^{-T} w            (transposed unit-lower solve)                 */
/*   gb  = P^T b'                                                            */
/*   dl/dU_ij = -sum_s w_is z_js   on the pattern of U (j >= i)             */
/*   dl/dL_ij = -sum_s b'_is y_js  on the strict lower pattern (j < i)      */
/* The gradients on the factor values are written in factor order (glu,    */
/* length nnz_lu, summed over the right-hand sides).                         */
/* ------------------------------------------------------------------------ */
void orc_adjoint(int n, const int *rp, const int *ci, const int *diag_pos, const double *val,
                 const int *perm, const double *gx, const double *x, const double *y, double *gb,
                 double *glu, int nrhs, long ld) {
    double *w = (double *)malloc(sizeof(double) * (size_t)n * (size_t)nrhs);
    double *bp = (double *)malloc(sizeof(double) * (size_t)n * (size_t)nrhs);
    for (int s = 0; s < nrhs; ++s) {
        double *ws = w + (size_t)s * n, *bs = bp + (size_t)s * n;
        for (int r = 0; r < n; ++r) ws[r] = gx[(long)perm[r] * ld + s];
        /* U^T w = P gx: rows of U are the columns of U^T; push form */
        for (int i = 0; i < n; ++i) {
            ws[i] = ws[i] / val[diag_pos[i]];
            for (int p = diag_pos[i] + 1; p < rp[i + 1]; ++p) {
                double prod = val[p] * ws[i];
                ws[ci[p]] = ws[ci[p]] - prod;
            }
        }
        /* L^T b' = w, unit diagonal, push form from the last row up */
        for (int i = 0; i < n; ++i) bs[i] = ws[i];
        for (int i = n - 1; i >= 0; --i) {
            for (int p = rp[i]; p < diag_pos[i]; ++p) {
                double prod = val[p] * bs[i];
                bs[ci[p]] = bs[ci[p]] - prod;
            }
        }
        for (int r = 0; r < n; ++r) gb[(long)perm[r] * ld + s] = bs[r];
    }
    for (int i = 0; i < n; ++i) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int j = ci[p];
            double acc = 0.0;
            for (int s = 0; s < nrhs; ++s) {
                double prod;
                if (j >= i) prod = w[(size_t)s * n + i] * x[(long)perm[j] * ld + s];
                else prod = bp[(size_t)s * n + i] * y[(long)j * ld + s];
                acc = acc + prod;
            }
            glu[p] = -acc;
        }
    }
    free(w);
    free(bp);
}
