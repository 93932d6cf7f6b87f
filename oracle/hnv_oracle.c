/*
 * FP64 CPU oracle for HyperNetVec multi-level refinement
 * (Maleki, Saless, Wall, Pingali, arXiv 2103.09660).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark (which also reports the GPU
 * results' errors against it) may load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * Conventions
 *   H = (V, E): hyperedges are sets of nodes (Section 1).  Input is the
 *   hyperedge->members CSR: eptr[n_edges+1] (int64), eidx[nnz] (int32), each
 *   row ascending without repeats; w[n_edges] float (NULL = unit weights).
 *   Star expansion H* (Section 1.1): one row per node and one per hyperedge,
 *   nodes first: row v for node v, row n_nodes+e for hyperedge e.  Embedding
 *   matrices are row-major double [rows x d].
 *
 * Every loop below runs rows independently and sums each row's terms in
 * ascending neighbour order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops below will use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops that follow (timing runs only). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Star-expansion neighbourhoods                                            */
/* ------------------------------------------------------------------------ */

/* Node -> incident hyperedges (the transpose of the member lists), each list
 * ascending in hyperedge id.  nptr[n_nodes+1], nidx[nnz] caller-allocated. */
void oracle_transpose(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                      const int32_t *eidx, int64_t *nptr, int32_t *nidx)
{
    int64_t *fill = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    memset(nptr, 0, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int64_t e = 0; e < n_edges; ++e)
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j)
            nptr[eidx[j] + 1] += 1;
    for (int64_t v = 0; v < n_nodes; ++v)
        nptr[v + 1] += nptr[v];
    for (int64_t e = 0; e < n_edges; ++e)
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j) {
            int32_t v = eidx[j];
            nidx[nptr[v] + fill[v]] = (int32_t)e;
            fill[v] += 1;
        }
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Coarsening, one level (Section 3.1, Algorithm 1, featureless variant)    */
/* ------------------------------------------------------------------------ */

/* Is hyperedge a a better assignment target than hyperedge b?  The paper
 * assigns a featureless node by hyperedge weight or degree; the reading used
 * here: heavier weight first, then fewer members, then the lower id (the
 * paper breaks ties at random; a fixed order keeps the maps reproducible). */
static int better_edge(int32_t a, int32_t b, const int64_t *eptr, const float *w)
{
    float wa = w ? w[a] : 1.0f, wb = w ? w[b] : 1.0f;
    if (wa != wb)
        return wa > wb;
    int64_t sa = eptr[a + 1] - eptr[a], sb = eptr[b + 1] - eptr[b];
    if (sa != sb)
        return sa < sb;
    return a < b;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Algorithm 1's steps after AssignHyperedge, given assigned[v] = c(v) (-1 for
 * an isolated node): FindAssignedNodes + Merge + addNode, addHedge, addEdge.
 * Outputs as for oracle_coarsen below. */
static void merge_assigned(int64_t n_nodes, int64_t n_edges, const int64_t *eptr, const int32_t *eidx,
                           const float *w, const int32_t *assigned, int32_t *group_id, int32_t *scratch,
                           int32_t *node_rep, int32_t *edge_rep, int64_t *out_nodes, int64_t *out_edges,
                           int64_t *out_nnz, int64_t *c_eptr, int32_t *c_eidx, float *c_w)
{
    /* The nodes assigned to one hyperedge become one coarse node; an
     * isolated node is its own group.  Coarse ids are issued in order of
     * each group's smallest fine node. */
    for (int64_t e = 0; e < n_edges; ++e)
        group_id[e] = -1;
    int32_t next = 0;
    for (int64_t v = 0; v < n_nodes; ++v) {
        int32_t e = assigned[v];
        if (e < 0) {
            node_rep[v] = next++;
        } else {
            if (group_id[e] < 0)
                group_id[e] = next++;
            node_rep[v] = group_id[e];
        }
    }
    *out_nodes = next;

    /* addHedge: hyperedge e survives unless every member was assigned to e. */
    int32_t n_keep = 0;
    for (int64_t e = 0; e < n_edges; ++e) {
        int64_t size = eptr[e + 1] - eptr[e], mine = 0;
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j)
            if (assigned[eidx[j]] == (int32_t)e)
                ++mine;
        edge_rep[e] = (mine == size) ? -1 : n_keep++;
    }
    *out_edges = n_keep;

    /* addEdge(rep(e), rep(v)) for v in e, as a set (duplicates collapse). */
    int64_t pos = 0;
    c_eptr[0] = 0;
    for (int64_t e = 0; e < n_edges; ++e) {
        if (edge_rep[e] < 0)
            continue;
        int64_t size = eptr[e + 1] - eptr[e];
        for (int64_t j = 0; j < size; ++j)
            scratch[j] = node_rep[eidx[eptr[e] + j]];
        qsort(scratch, (size_t)size, sizeof(int32_t), cmp_i32);
        int64_t kept = 0;
        for (int64_t j = 0; j < size; ++j)
            if (kept == 0 || scratch[j] != c_eidx[pos + kept - 1])
                c_eidx[pos + kept++] = scratch[j];
        pos += kept;
        c_eptr[edge_rep[e] + 1] = pos;
        if (c_w)
            c_w[edge_rep[e]] = w ? w[e] : 1.0f;
    }
    *out_nnz = pos;
}

/* One application of Algorithm 1's loop body without features.
 *   node_rep[n_nodes]   coarse node of each fine node (rep(v))
 *   edge_rep[n_edges]   coarse hyperedge of each fine hyperedge, -1 if removed
 *   c_eptr[n_edges+1], c_eidx[nnz], c_w[n_edges]: coarse CSR (sizes bounded
 *   by the fine ones); *out_nodes, *out_edges, *out_nnz receive the sizes.
 * Returns 0, or -1 if memory ran out. */
int oracle_coarsen(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                   const int32_t *eidx, const float *w, int32_t *node_rep,
                   int32_t *edge_rep, int64_t *out_nodes, int64_t *out_edges,
                   int64_t *out_nnz, int64_t *c_eptr, int32_t *c_eidx, float *c_w)
{
    int64_t nnz = eptr[n_edges];
    int64_t *nptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int32_t *nidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *assigned = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    int32_t *group_id = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_edges > 0 ? n_edges : 1));
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!nptr || !nidx || !assigned || !group_id || !scratch) {
        free(nptr); free(nidx); free(assigned); free(group_id); free(scratch);
        return -1;
    }
    oracle_transpose(n_nodes, n_edges, eptr, eidx, nptr, nidx);

    /* AssignHyperedge: c(v) = best hyperedge in N(v); none for isolated v. */
    for (int64_t v = 0; v < n_nodes; ++v) {
        int32_t best = -1;
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int32_t e = nidx[j];
            if (best < 0 || better_edge(e, best, eptr, w))
                best = e;
        }
        assigned[v] = best;
    }
    merge_assigned(n_nodes, n_edges, eptr, eidx, w, assigned, group_id, scratch, node_rep, edge_rep, out_nodes,
                   out_edges, out_nnz, c_eptr, c_eidx, c_w);
    free(nptr); free(nidx); free(assigned); free(group_id); free(scratch);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Coarsening, one level, with node features (Section 3.1, Algorithm 1)     */
/* ------------------------------------------------------------------------ */

/* The cosine score of hyperedge e for node v, as the value the argmax is
 * taken on.  f(e) is the mean of the member features (ComputeEdgeFeature);
 * the cosine of f(e) and f(v) equals d / (|s_e| |x_v|) with s_e the member
 * sum, d = s_e . x_v, because the factor 1/|e| cancels.  The features are
 * bag-of-words counts, so d and |s_e|^2 are exact integers.  For a fixed v
 * the value q = d |d| / |s_e|^2 equals cos |cos| |x_v|^2, an increasing
 * function of the cosine; it is evaluated in IEEE FP64 (one product, one
 * quotient, each rounded once).  q = 0 when s_e = 0 (the cosine is then
 * undefined and no hyperedge is preferred on features). */
static double cosine_score(int64_t d, int64_t s2)
{
    if (s2 == 0)
        return 0.0;
    double dd = (double)d;
    double num = dd * fabs(dd);
    return num / (double)s2;
}

/* Algorithm 1's loop body once with node features X [n_nodes x k] (int32
 * counts, >= 0, total below 2^31).
 *   ComputeEdgeFeature: s_e = sum of member rows (the mean up to 1/|e|).
 *   AssignHyperedge:    c(v) = argmax over e in N(v) of the cosine of f(e)
 *                       and f(v); equal scores are broken by the featureless
 *                       order (heavier, then fewer members, then lower id),
 *                       in place of the paper's random choice.
 *   Merge etc.:         as without features.
 *   X':                 each coarse node's row is the sum of its fine
 *                       nodes' rows (the merged bags of words).
 * Other arguments as oracle_coarsen; c_x[n_nodes x k] receives X' (the
 * first *out_nodes rows).  Returns 0, or -1 if memory ran out. */
int oracle_coarsen_features(int64_t n_nodes, int64_t n_edges, const int64_t *eptr, const int32_t *eidx,
                            const float *w, const int32_t *x, int k, int32_t *node_rep, int32_t *edge_rep,
                            int64_t *out_nodes, int64_t *out_edges, int64_t *out_nnz, int64_t *c_eptr,
                            int32_t *c_eidx, float *c_w, int32_t *c_x)
{
    int64_t nnz = eptr[n_edges];
    int64_t *nptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int32_t *nidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *assigned = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    int32_t *group_id = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_edges > 0 ? n_edges : 1));
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    /* member sums fit int32: the counts total below 2^31 */
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_edges > 0 ? n_edges : 1) * (size_t)k);
    int64_t *s2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_edges > 0 ? n_edges : 1));
    if (!nptr || !nidx || !assigned || !group_id || !scratch || !s || !s2) {
        free(nptr); free(nidx); free(assigned); free(group_id); free(scratch); free(s); free(s2);
        return -1;
    }
    oracle_transpose(n_nodes, n_edges, eptr, eidx, nptr, nidx);

    /* ComputeEdgeFeature for every hyperedge, and |s_e|^2. */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t *se = s + (size_t)e * k;
        for (int j = 0; j < k; ++j)
            se[j] = 0;
        for (int64_t m = eptr[e]; m < eptr[e + 1]; ++m) {
            const int32_t *xv = x + (size_t)eidx[m] * k;
            for (int j = 0; j < k; ++j)
                se[j] += xv[j];
        }
        int64_t q = 0;
        for (int j = 0; j < k; ++j)
            q += (int64_t)se[j] * se[j];
        s2[e] = q;
    }

    /* AssignHyperedge: the best cosine over N(v), ties by the fixed order. */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_nodes; ++v) {
        const int32_t *xv = x + (size_t)v * k;
        int32_t best = -1;
        double best_q = 0.0;
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int32_t e = nidx[j];
            const int32_t *se = s + (size_t)e * k;
            int64_t d = 0;
            for (int c = 0; c < k; ++c)
                d += (int64_t)se[c] * xv[c];
            double q = cosine_score(d, s2[e]);
            if (best < 0 || q > best_q || (q == best_q && better_edge(e, best, eptr, w))) {
                best = e;
                best_q = q;
            }
        }
        assigned[v] = best;
    }
    merge_assigned(n_nodes, n_edges, eptr, eidx, w, assigned, group_id, scratch, node_rep, edge_rep, out_nodes,
                   out_edges, out_nnz, c_eptr, c_eidx, c_w);

    /* X': the merged nodes' rows summed (int32 suffices: the counts total
     * below 2^31). */
    memset(c_x, 0, sizeof(int32_t) * (size_t)*out_nodes * (size_t)k);
    for (int64_t v = 0; v < n_nodes; ++v) {
        int32_t *dst = c_x + (size_t)node_rep[v] * k;
        const int32_t *xv = x + (size_t)v * k;
        for (int j = 0; j < k; ++j)
            dst[j] += xv[j];
    }
    free(nptr); free(nidx); free(assigned); free(group_id); free(scratch); free(s); free(s2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection (Section 3.3, last paragraph before the SOR remark)           */
/* ------------------------------------------------------------------------ */

/* Row map from the fine star expansion to the coarse one.  A fine node takes
 * the row of the coarse node it was merged into.  A kept hyperedge takes the
 * row of rep(e).  A removed hyperedge had all of its members merged into one
 * coarse node and takes that node's row. */
void oracle_rowmap(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                   const int32_t *eidx, const int32_t *node_rep,
                   const int32_t *edge_rep, int64_t n_nodes_coarse, int64_t *rowmap)
{
    for (int64_t v = 0; v < n_nodes; ++v)
        rowmap[v] = node_rep[v];
    for (int64_t e = 0; e < n_edges; ++e) {
        if (edge_rep[e] >= 0)
            rowmap[n_nodes + e] = n_nodes_coarse + edge_rep[e];
        else
            rowmap[n_nodes + e] = node_rep[eidx[eptr[e]]];
    }
}

void oracle_project(int64_t rows_fine, const int64_t *rowmap, int64_t d,
                    const double *zc, double *zf)
{
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < rows_fine; ++u)
        memcpy(zf + u * d, zc + rowmap[u] * d, sizeof(double) * (size_t)d);
}

/* ------------------------------------------------------------------------ */
/* Refinement sweep (Algorithm 2, one iteration of the while loop)          */
/* ------------------------------------------------------------------------ */

/* z_out[u] = (1 - omega) z_src[u] + omega * (sum_v w_uv z_nb[v]) / (sum_v w_uv)
 * over the star-expansion neighbours v of row u, where the weight of the star
 * edge between node v and hyperedge e is w_e in both directions.  A row with
 * no neighbours keeps its value.  d doubles accumulate per row in `acc`. */
static void relax_row(int64_t u_row, const int64_t *ptr, const int32_t *nb, int64_t nb_base,
                      int64_t self, const float *w_of_nb, float w_self, int use_self_w,
                      int64_t d, double omega, const double *z_src, const double *z_nb,
                      double *z_out, double *acc)
{
    double den = 0.0;
    for (int64_t c = 0; c < d; ++c)
        acc[c] = 0.0;
    for (int64_t j = ptr[u_row]; j < ptr[u_row + 1]; ++j) {
        int64_t v = nb[j];
        double wuv = use_self_w ? (double)w_self : (w_of_nb ? (double)w_of_nb[v] : 1.0);
        den += wuv;
        const double *zv = z_nb + (nb_base + v) * d;
        for (int64_t c = 0; c < d; ++c)
            acc[c] += wuv * zv[c];
    }
    const double *zu = z_src + self * d;
    double *out = z_out + self * d;
    if (den == 0.0) {
        for (int64_t c = 0; c < d; ++c)
            out[c] = zu[c];
    } else {
        for (int64_t c = 0; c < d; ++c)
            out[c] = (1.0 - omega) * zu[c] + omega * (acc[c] / den);
    }
}

/* order 0: every row reads z_in (the pseudocode's z^{i-1} on every right-hand
 * side).  order 1: hyperedge rows first from the old node rows, then node
 * rows from the new hyperedge rows.  nptr/nidx is the transpose of eptr/eidx.
 * z_in and z_out must not alias. */
void oracle_sweep(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                  const int32_t *eidx, const int64_t *nptr, const int32_t *nidx,
                  const float *w, int64_t d, double omega, int order,
                  const double *z_in, double *z_out)
{
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)d);
        /* hyperedge rows: neighbours are the member nodes, weight w_e */
#pragma omp for schedule(dynamic, 256)
        for (int64_t e = 0; e < n_edges; ++e)
            relax_row(e, eptr, eidx, 0, n_nodes + e, NULL, w ? w[e] : 1.0f, 1, d, omega,
                      z_in, z_in, z_out, acc);
        /* node rows: neighbours are the incident hyperedges, weight w_e */
        const double *z_nb = (order == 1) ? z_out : z_in;
#pragma omp for schedule(dynamic, 256)
        for (int64_t v = 0; v < n_nodes; ++v)
            relax_row(v, nptr, nidx, n_nodes, v, w, 0.0f, 0, d, omega, z_in, z_nb, z_out, acc);
        free(acc);
    }
}

/* ------------------------------------------------------------------------ */
/* Reverse mode of one order-0 sweep                                        */
/* ------------------------------------------------------------------------ */

/* Given y = z^{i-1}, g = dL/dz^i, writes gy = dL/dy and adds dL/dw_e into
 * dw[n_edges] (if dw != NULL).  Derived from the forward rule above:
 *   node v with S_v = sum_{e ∋ v} w_e > 0:
 *       z_v = (1-omega) y_v + omega sum_{e ∋ v} (w_e / S_v) y_e
 *   hyperedge e with |e| > 0 (its weight cancels):
 *       z_e = (1-omega) y_e + omega sum_{v ∈ e} (1 / |e|) y_v
 *   empty rows: z = y.
 * Hence
 *   gy_v = s_v g_v + omega sum_{e ∋ v} g_e / |e|         (s = 1-omega, or 1 if empty)
 *   gy_e = s_e g_e + omega sum_{v ∈ e} (w_e / S_v) g_v
 *   dL/dw_e = omega sum_{v ∈ e} <g_v, y_e - ztilde_v> / S_v,
 *             ztilde_v = sum_{e' ∋ v} w_e' y_e' / S_v. */
void oracle_sweep_vjp(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                      const int32_t *eidx, const int64_t *nptr, const int32_t *nidx,
                      const float *w, int64_t d, double omega, const double *y,
                      const double *g, double *gy, double *dw)
{
    double *S = (double *)malloc(sizeof(double) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    double *zt = (double *)malloc(sizeof(double) * (size_t)(n_nodes > 0 ? n_nodes : 1) * (size_t)d);
    /* per node: S_v and ztilde_v */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_nodes; ++v) {
        double s = 0.0;
        double *t = zt + v * d;
        for (int64_t c = 0; c < d; ++c)
            t[c] = 0.0;
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int64_t e = nidx[j];
            double we = w ? (double)w[e] : 1.0;
            s += we;
            for (int64_t c = 0; c < d; ++c)
                t[c] += we * y[(n_nodes + e) * d + c];
        }
        S[v] = s;
        if (s != 0.0)
            for (int64_t c = 0; c < d; ++c)
                t[c] /= s;
    }
    /* node rows of gy */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_nodes; ++v) {
        double self = (nptr[v + 1] > nptr[v]) ? 1.0 - omega : 1.0;
        for (int64_t c = 0; c < d; ++c)
            gy[v * d + c] = self * g[v * d + c];
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int64_t e = nidx[j];
            double size = (double)(eptr[e + 1] - eptr[e]);
            for (int64_t c = 0; c < d; ++c)
                gy[v * d + c] += omega * g[(n_nodes + e) * d + c] / size;
        }
    }
    /* hyperedge rows of gy, and the weight gradient */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < n_edges; ++e) {
        int64_t row = n_nodes + e;
        double we = w ? (double)w[e] : 1.0;
        double self = (eptr[e + 1] > eptr[e]) ? 1.0 - omega : 1.0;
        double gw = 0.0;
        for (int64_t c = 0; c < d; ++c)
            gy[row * d + c] = self * g[row * d + c];
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j) {
            int64_t v = eidx[j];
            double dot = 0.0;
            for (int64_t c = 0; c < d; ++c) {
                gy[row * d + c] += omega * (we / S[v]) * g[v * d + c];
                dot += g[v * d + c] * (y[row * d + c] - zt[v * d + c]);
            }
            gw += omega * dot / S[v];
        }
        if (dw)
            dw[e] += gw;
    }
    free(S);
    free(zt);
}

/* Reverse mode of one edge-first sweep (Section 3.3's reading as two
 * partial relaxations: hyperedge rows from the old node rows, then node rows
 * from the new hyperedge rows).  With y the sweep's input and g = dL/dZ':
 *   e'_e  = (1-omega) y_e + omega mean_{v in e} y_v      (the new hyperedge rows)
 *   zt_v  = sum_{e ∋ v} w_e e'_e / S_v,  S_v = sum_{e ∋ v} w_e
 * the node half gives
 *   dL/dy_v  = (1-omega) g_v            (g_v for a node without hyperedges)
 *   dL/de'_e = g_e + omega w_e sum_{v in e} g_v / S_v
 *   dL/dw_e += omega sum_{v in e} <g_v, e'_e - zt_v> / S_v
 * and the hyperedge half then adds
 *   dL/dy_e  = (1-omega) dL/de'_e
 *   dL/dy_v += omega sum_{e ∋ v} dL/de'_e / |e|.
 * Every hyperedge has members, so every hyperedge row is relaxed. */
void oracle_sweep_vjp_edge_first(int64_t n_nodes, int64_t n_edges, const int64_t *eptr,
                                 const int32_t *eidx, const int64_t *nptr, const int32_t *nidx,
                                 const float *w, int64_t d, double omega, const double *y,
                                 const double *g, double *gy, double *dw)
{
    const size_t ne = (size_t)(n_edges > 0 ? n_edges : 1), nv = (size_t)(n_nodes > 0 ? n_nodes : 1);
    double *ep = (double *)malloc(sizeof(double) * ne * (size_t)d);   /* e' */
    double *gep = (double *)malloc(sizeof(double) * ne * (size_t)d);  /* dL/de' */
    double *S = (double *)malloc(sizeof(double) * nv);
    double *zt = (double *)malloc(sizeof(double) * nv * (size_t)d);
    /* the hyperedge half of the forward sweep */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < n_edges; ++e) {
        const double size = (double)(eptr[e + 1] - eptr[e]);
        for (int64_t c = 0; c < d; ++c) {
            double m = 0.0;
            for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j)
                m += y[(int64_t)eidx[j] * d + c];
            ep[e * d + c] = (1.0 - omega) * y[(n_nodes + e) * d + c] + omega * m / size;
        }
    }
    /* per node: S_v and the weighted mean of its new hyperedge rows */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_nodes; ++v) {
        double s = 0.0;
        double *t = zt + v * d;
        for (int64_t c = 0; c < d; ++c)
            t[c] = 0.0;
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int64_t e = nidx[j];
            double we = w ? (double)w[e] : 1.0;
            s += we;
            for (int64_t c = 0; c < d; ++c)
                t[c] += we * ep[e * d + c];
        }
        S[v] = s;
        if (s != 0.0)
            for (int64_t c = 0; c < d; ++c)
                t[c] /= s;
    }
    /* the node half in reverse: dL/de' and the weight gradient per hyperedge */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < n_edges; ++e) {
        double we = w ? (double)w[e] : 1.0;
        double gw = 0.0;
        for (int64_t c = 0; c < d; ++c)
            gep[e * d + c] = g[(n_nodes + e) * d + c];
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j) {
            int64_t v = eidx[j];
            double dot = 0.0;
            for (int64_t c = 0; c < d; ++c) {
                gep[e * d + c] += omega * (we / S[v]) * g[v * d + c];
                dot += g[v * d + c] * (ep[e * d + c] - zt[v * d + c]);
            }
            gw += omega * dot / S[v];
        }
        if (dw)
            dw[e] += gw;
        for (int64_t c = 0; c < d; ++c)
            gy[(n_nodes + e) * d + c] = (1.0 - omega) * gep[e * d + c];
    }
    /* node rows: their own term from the node half, then the hyperedge half */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_nodes; ++v) {
        double self = (nptr[v + 1] > nptr[v]) ? 1.0 - omega : 1.0;
        for (int64_t c = 0; c < d; ++c)
            gy[v * d + c] = self * g[v * d + c];
        for (int64_t j = nptr[v]; j < nptr[v + 1]; ++j) {
            int64_t e = nidx[j];
            double size = (double)(eptr[e + 1] - eptr[e]);
            for (int64_t c = 0; c < d; ++c)
                gy[v * d + c] += omega * gep[e * d + c] / size;
        }
    }
    free(ep);
    free(gep);
    free(S);
    free(zt);
}

/* Reverse mode of the projection: every fine row's gradient is added to the
 * coarse row it was copied from, in ascending fine-row order. */
void oracle_project_vjp(int64_t rows_fine, int64_t rows_coarse, const int64_t *rowmap,
                        int64_t d, const double *gf, double *gc)
{
    memset(gc, 0, sizeof(double) * (size_t)(rows_coarse * d));
    for (int64_t u = 0; u < rows_fine; ++u)
        for (int64_t c = 0; c < d; ++c)
            gc[rowmap[u] * d + c] += gf[u * d + c];
}
