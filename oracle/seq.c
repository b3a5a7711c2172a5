/*
 * Oracle (test infrastructure only): the sequential integer steps of the
 * multigrid setup and the ordered Galerkin sums, written as plain loops.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the GPU library.  Built with
 * -O2 -ffp-contract=off so every product and sum is one IEEE rounding, in the
 * order the loops state.
 *
 *  or_aggregate  : distance-2 maximal independent set by sequential greedy in
 *                  descending key order, then the two aggregation phases
 *                  (Sec. 4.3.1: disjoint aggregates covering every node, one
 *                  coarse node per aggregate).
 *  or_colour     : first-fit greedy colouring in increasing node order.
 *  or_rap_stage1 : T = A P for piecewise-constant P (per fine row, grouped by
 *                  the aggregate of the column node).
 *  or_rap_stage2 : A_c = P^T T (per aggregate, members in increasing order).
 *                  Together: the Galerkin product of Sec. 3 with R = P^T.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t key; int32_t node; } keyed_t;

static int cmp_desc(const void* a, const void* b) {
    uint64_t ka = ((const keyed_t*)a)->key, kb = ((const keyed_t*)b)->key;
    return (ka < kb) - (ka > kb);
}

/* Strong graph in CSR (symmetric, no self loops), squared edge weights w2.
 * key[i] gives the priority (larger first).  Writes agg[i] in [0, n_agg).
 * Returns 0 on success, -1 if some node could not be attached (only possible
 * if the graph is not symmetric). */
int or_aggregate(int n, const int32_t* ptr, const int32_t* idx, const double* w2,
                 const uint64_t* key, int32_t* agg, int32_t* n_agg_out) {
    keyed_t* order = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* covered = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t* is_root = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t* root_id = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* phase1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int rc = 0;
    for (int i = 0; i < n; ++i) { order[i].key = key[i]; order[i].node = i; }
    qsort(order, (size_t)n, sizeof(keyed_t), cmp_desc);
    /* Greedy distance-2 MIS: a node becomes a root iff no root lies within two hops. */
    for (int t = 0; t < n; ++t) {
        int v = order[t].node;
        if (covered[v]) continue;
        is_root[v] = 1;
        covered[v] = 1;
        for (int p = ptr[v]; p < ptr[v + 1]; ++p) {
            int u = idx[p];
            covered[u] = 1;
            for (int q = ptr[u]; q < ptr[u + 1]; ++q) covered[idx[q]] = 1;
        }
    }
    /* Aggregate ids ordered by root node index. */
    int n_agg = 0;
    for (int i = 0; i < n; ++i) root_id[i] = is_root[i] ? n_agg++ : -1;
    /* Phase 1: each root with its strong neighbours. */
    for (int i = 0; i < n; ++i) phase1[i] = -1;
    for (int i = 0; i < n; ++i) {
        if (!is_root[i]) continue;
        phase1[i] = root_id[i];
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) phase1[idx[p]] = root_id[i];
    }
    /* Phase 2: every other node joins the phase-1 aggregate of its strongest
     * assigned neighbour; equal weights go to the smaller aggregate id. */
    for (int i = 0; i < n; ++i) {
        if (phase1[i] >= 0) { agg[i] = phase1[i]; continue; }
        int best = -1;
        double bw = 0.0;
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            int a = phase1[idx[p]];
            if (a < 0) continue;
            if (best < 0 || w2[p] > bw || (w2[p] == bw && a < best)) { best = a; bw = w2[p]; }
        }
        if (best < 0) { rc = -1; best = 0; }
        agg[i] = best;
    }
    *n_agg_out = n_agg;
    free(order); free(covered); free(is_root); free(root_id); free(phase1);
    return rc;
}

/* First-fit greedy colouring, nodes in increasing index, over a symmetric
 * pattern (self entries ignored).  Returns the number of colours. */
int or_colour(int n, const int32_t* ptr, const int32_t* idx, int32_t* colour) {
    int ncol = 0;
    int cap = 64;
    int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    for (int c = 0; c < cap; ++c) mark[c] = -1;
    for (int i = 0; i < n; ++i) colour[i] = -1;
    for (int i = 0; i < n; ++i) {
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            int j = idx[p];
            if (j == i || colour[j] < 0) continue;
            mark[colour[j]] = i;
        }
        int c = 0;
        while (c < cap && mark[c] == i) ++c;
        if (c == cap) {
            int ncap = cap * 2;
            mark = (int32_t*)realloc(mark, sizeof(int32_t) * (size_t)ncap);
            for (int k = cap; k < ncap; ++k) mark[k] = -1;
            cap = ncap;
        }
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(mark);
    return ncol;
}

/* Stage 1: T = A * P with P[(j,c),(agg[j],c)] = qc[j*bc+c].
 * A in BSR (br x bc blocks, columns sorted).  T row i lists the distinct
 * aggregates of its column nodes in increasing order; each entry sums
 * A_ij[r,c]*qc[j,c] over the row's columns j in increasing order.
 * Output arrays sized by the caller to at least nnzb(A).  Returns nnzb(T). */
int64_t or_rap_stage1(int n, int br, int bc, const int32_t* rp, const int32_t* ci,
                      const double* val, const int32_t* agg, const double* qc,
                      int32_t* t_rp, int32_t* t_ci, double* t_val) {
    int64_t nz = 0;
    int bs = br * bc;
    t_rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        int64_t row_start = nz;
        /* distinct aggregates of the row, sorted */
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int l = agg[ci[p]];
            int64_t q = row_start;
            while (q < nz && t_ci[q] < l) ++q;
            if (q < nz && t_ci[q] == l) continue;
            for (int64_t s = nz; s > q; --s) t_ci[s] = t_ci[s - 1];
            t_ci[q] = l;
            ++nz;
        }
        for (int64_t q = row_start; q < nz; ++q) {
            double* acc = t_val + q * bs;
            for (int k = 0; k < bs; ++k) acc[k] = 0.0;
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                int j = ci[p];
                if (agg[j] != t_ci[q]) continue;
                const double* a = val + (int64_t)p * bs;
                for (int r = 0; r < br; ++r)
                    for (int c = 0; c < bc; ++c) {
                        double term = a[r * bc + c] * qc[(int64_t)j * bc + c];
                        acc[r * bc + c] = acc[r * bc + c] + term;
                    }
            }
        }
        t_rp[i + 1] = (int32_t)nz;
    }
    return nz;
}

/* Stage 2: C = P^T T with P[(i,r),(agg[i],r)] = qr[i*br+r].
 * Aggregate k's members given in increasing order by (m_ptr, m_idx).
 * Each coarse entry sums qr[i,r]*T[i,l][r,c] over members i in order.
 * Output arrays sized by the caller to at least nnzb(T).  Returns nnzb(C). */
int64_t or_rap_stage2(int nc, int br, int bc, const int32_t* m_ptr, const int32_t* m_idx,
                      const int32_t* t_rp, const int32_t* t_ci, const double* t_val,
                      const double* qr, int32_t* c_rp, int32_t* c_ci, double* c_val) {
    int64_t nz = 0;
    int bs = br * bc;
    c_rp[0] = 0;
    for (int k = 0; k < nc; ++k) {
        int64_t row_start = nz;
        for (int m = m_ptr[k]; m < m_ptr[k + 1]; ++m) {
            int i = m_idx[m];
            for (int p = t_rp[i]; p < t_rp[i + 1]; ++p) {
                int l = t_ci[p];
                int64_t q = row_start;
                while (q < nz && c_ci[q] < l) ++q;
                if (q < nz && c_ci[q] == l) continue;
                for (int64_t s = nz; s > q; --s) c_ci[s] = c_ci[s - 1];
                c_ci[q] = l;
                ++nz;
            }
        }
        for (int64_t q = row_start; q < nz; ++q) {
            double* acc = c_val + q * bs;
            for (int e = 0; e < bs; ++e) acc[e] = 0.0;
            for (int m = m_ptr[k]; m < m_ptr[k + 1]; ++m) {
                int i = m_idx[m];
                for (int p = t_rp[i]; p < t_rp[i + 1]; ++p) {
                    if (t_ci[p] != c_ci[q]) continue;
                    const double* t = t_val + (int64_t)p * bs;
                    for (int r = 0; r < br; ++r)
                        for (int c = 0; c < bc; ++c) {
                            double term = qr[(int64_t)i * br + r] * t[r * bc + c];
                            acc[r * bc + c] = acc[r * bc + c] + term;
                        }
                }
            }
        }
        c_rp[k + 1] = (int32_t)nz;
    }
    return nz;
}

/* C = A B for block-sparse A (n rows, br x bm blocks) and B (bm x bc blocks),
 * rows of both with increasing columns.  Row i of C lists the distinct columns
 * reached through row i of A in increasing order; entry (r,c) of block (i,l)
 * sums A[i,j][r][m] * B[j,l][m][c] over the columns j of row i in increasing
 * order and, for each j, over m in increasing order.  With B the
 * piecewise-constant prolongator this is exactly or_rap_stage1, and with A
 * its transpose it is or_rap_stage2.  Output arrays sized by the caller
 * (cap blocks).  Returns nnzb(C), or -1 when cap is too small. */
int64_t or_spgemm(int n, int br, int bm, int bc, const int32_t* a_rp, const int32_t* a_ci, const double* a_val,
                  const int32_t* b_rp, const int32_t* b_ci, const double* b_val, int64_t cap,
                  int32_t* c_rp, int32_t* c_ci, double* c_val) {
    int64_t nz = 0;
    const int as = br * bm, bs = bm * bc, cs = br * bc;
    c_rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        int64_t row_start = nz;
        for (int p = a_rp[i]; p < a_rp[i + 1]; ++p) {
            int j = a_ci[p];
            for (int q = b_rp[j]; q < b_rp[j + 1]; ++q) {
                int l = b_ci[q];
                int64_t s = row_start;
                while (s < nz && c_ci[s] < l) ++s;
                if (s < nz && c_ci[s] == l) continue;
                if (nz >= cap) return -1;
                for (int64_t t = nz; t > s; --t) c_ci[t] = c_ci[t - 1];
                c_ci[s] = l;
                ++nz;
            }
        }
        for (int64_t s = row_start; s < nz; ++s) {
            double* acc = c_val + s * cs;
            for (int e = 0; e < cs; ++e) acc[e] = 0.0;
            for (int p = a_rp[i]; p < a_rp[i + 1]; ++p) {
                int j = a_ci[p];
                for (int q = b_rp[j]; q < b_rp[j + 1]; ++q) {
                    if (b_ci[q] != c_ci[s]) continue;
                    const double* a = a_val + (int64_t)p * as;
                    const double* b = b_val + (int64_t)q * bs;
                    for (int r = 0; r < br; ++r)
                        for (int c = 0; c < bc; ++c)
                            for (int m = 0; m < bm; ++m) {
                                double term = a[r * bm + m] * b[m * bc + c];
                                acc[r * bc + c] = acc[r * bc + c] + term;
                            }
                }
            }
        }
        c_rp[i + 1] = (int32_t)nz;
    }
    return nz;
}

/* Smoothed prolongator of one block (vector components only):
 *   P = Phat - D_vv^-1 A_vv Phat W
 * with Phat[(i,a),(agg(i),a)] = q[i,a], D_vv the diagonal of the vector-vector
 * part of A_ff, W = diag(w) over coarse nodes.  Row i lists, in increasing
 * order, agg(i) and the aggregates k of its columns with w[k] != 0 (a zero
 * weight adds nothing outside the node's own aggregate, so w = 0 gives Phat
 * exactly, pattern included).  For vector row a and vector
 * column c of block (i,k):
 *   s = sum over columns j of row i in increasing order with agg(j) = k of A[i,j][a][c] * q[j,c]
 *   P = base - w[k] * (s / A[i,i][a][a]),  base = q[i,a] if (k = agg(i), c = a) else 0
 * other entries are base.  Returns nnzb(P); output arrays hold nnzb(A) blocks. */
int64_t or_sa_prolongator(int n, int d, int nv, const int32_t* rp, const int32_t* ci, const double* val,
                          const int32_t* agg, const double* q, const double* w,
                          int32_t* p_rp, int32_t* p_ci, double* p_val) {
    int64_t nz = 0;
    const int bs = d * d;
    p_rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        int64_t row_start = nz;
        int pd = -1;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] == i) pd = p;
            int l = agg[ci[p]];
            if (l != agg[i] && w[l] == 0.0) continue;
            int64_t s = row_start;
            while (s < nz && p_ci[s] < l) ++s;
            if (s < nz && p_ci[s] == l) continue;
            for (int64_t t = nz; t > s; --t) p_ci[t] = p_ci[t - 1];
            p_ci[s] = l;
            ++nz;
        }
        for (int64_t s = row_start; s < nz; ++s) {
            int k = p_ci[s];
            double* out = p_val + s * bs;
            for (int a = 0; a < d; ++a)
                for (int c = 0; c < d; ++c) {
                    double base = (k == agg[i] && c == a) ? q[(int64_t)i * d + a] : 0.0;
                    if (a < nv && c < nv) {
                        double acc = 0.0;
                        for (int p = rp[i]; p < rp[i + 1]; ++p) {
                            int j = ci[p];
                            if (agg[j] != k) continue;
                            double term = val[(int64_t)p * bs + a * d + c] * q[(int64_t)j * d + c];
                            acc = acc + term;
                        }
                        double dg = val[(int64_t)pd * bs + a * d + a];
                        double t = acc / dg;
                        double u = w[k] * t;
                        out[a * d + c] = base - u;
                    } else {
                        out[a * d + c] = base;
                    }
                }
        }
        p_rp[i + 1] = (int32_t)nz;
    }
    return nz;
}
