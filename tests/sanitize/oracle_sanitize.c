/* Address / undefined-behaviour sanitizer run of the FP64 oracle (test
 * infrastructure): every entry point on seeded random hypergraphs with
 * isolated nodes and singleton hyperedges, three coarsening steps, both
 * sweep orders, the reverse mode and the feature-driven coarsening.  Built
 * with gcc -fsanitize=address,undefined by tests/test_sanitizers.py; any
 * report aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_coarsen(int64_t, int64_t, const int64_t *, const int32_t *, const float *, int32_t *, int32_t *,
                   int64_t *, int64_t *, int64_t *, int64_t *, int32_t *, float *);
int oracle_coarsen_features(int64_t, int64_t, const int64_t *, const int32_t *, const float *, const int32_t *,
                            int, int32_t *, int32_t *, int64_t *, int64_t *, int64_t *, int64_t *, int32_t *,
                            float *, int32_t *);
void oracle_transpose(int64_t, int64_t, const int64_t *, const int32_t *, int64_t *, int32_t *);
void oracle_rowmap(int64_t, int64_t, const int64_t *, const int32_t *, const int32_t *, const int32_t *, int64_t,
                   int64_t *);
void oracle_project(int64_t, const int64_t *, int64_t, const double *, double *);
void oracle_sweep(int64_t, int64_t, const int64_t *, const int32_t *, const int64_t *, const int32_t *,
                  const float *, int64_t, double, int, const double *, double *);
void oracle_sweep_vjp(int64_t, int64_t, const int64_t *, const int32_t *, const int64_t *, const int32_t *,
                      const float *, int64_t, double, const double *, const double *, double *, double *);
void oracle_project_vjp(int64_t, int64_t, const int64_t *, int64_t, const double *, double *);

static uint64_t state = 88172645463325252ull;
static uint32_t next(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 16);
}

static int cmp(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* random hypergraph: member sets of 1..max_size distinct nodes, ascending */
static void make(int64_t n, int64_t m, int max_size, int64_t **eptr, int32_t **eidx, float **w)
{
    *eptr = malloc(sizeof(int64_t) * (size_t)(m + 1));
    *eidx = malloc(sizeof(int32_t) * (size_t)(m * max_size + 1));
    *w = malloc(sizeof(float) * (size_t)(m + 1));
    (*eptr)[0] = 0;
    for (int64_t e = 0; e < m; ++e) {
        int size = 1 + (int)(next() % (uint32_t)max_size);
        if (size > n)
            size = (int)n;
        int32_t *row = *eidx + (*eptr)[e];
        int k = 0;
        while (k < size) {
            int32_t v = (int32_t)(next() % (uint32_t)n), dup = 0;
            for (int i = 0; i < k; ++i)
                dup |= row[i] == v;
            if (!dup)
                row[k++] = v;
        }
        qsort(row, (size_t)size, sizeof(int32_t), cmp);
        (*eptr)[e + 1] = (*eptr)[e] + size;
        (*w)[e] = (float)(1 + next() % 3);
    }
}

static int one_case(int64_t n, int64_t m, int max_size, int64_t d)
{
    int64_t *eptr;
    int32_t *eidx;
    float *w;
    make(n, m, max_size, &eptr, &eidx, &w);
    for (int step = 0; step < 3; ++step) {
        int64_t nnz = eptr[m], rows = n + m;
        int32_t *nrep = malloc(sizeof(int32_t) * (size_t)(n + 1)), *erep = malloc(sizeof(int32_t) * (size_t)(m + 1));
        int64_t *ceptr = malloc(sizeof(int64_t) * (size_t)(m + 1));
        int32_t *ceidx = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
        float *cw = malloc(sizeof(float) * (size_t)(m + 1));
        int64_t cn = 0, cm = 0, cz = 0;
        if (oracle_coarsen(n, m, eptr, eidx, w, nrep, erep, &cn, &cm, &cz, ceptr, ceidx, cw) != 0)
            return 1;
        /* features: the same step driven by small word counts */
        const int k = 8;
        int32_t *x = malloc(sizeof(int32_t) * (size_t)(n * k + 1)), *cx = malloc(sizeof(int32_t) * (size_t)(n * k + 1));
        for (int64_t i = 0; i < n * k; ++i)
            x[i] = (int32_t)(next() % 4 == 0 ? next() % 3 : 0);
        int32_t *fnrep = malloc(sizeof(int32_t) * (size_t)(n + 1)), *ferep = malloc(sizeof(int32_t) * (size_t)(m + 1));
        int64_t *feptr = malloc(sizeof(int64_t) * (size_t)(m + 1));
        int32_t *feidx = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
        float *fw = malloc(sizeof(float) * (size_t)(m + 1));
        int64_t fn = 0, fm = 0, fz = 0;
        if (oracle_coarsen_features(n, m, eptr, eidx, w, x, k, fnrep, ferep, &fn, &fm, &fz, feptr, feidx, fw, cx) != 0)
            return 1;
        /* sweeps, both orders, and the reverse mode */
        int64_t *nptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t *nidx = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
        oracle_transpose(n, m, eptr, eidx, nptr, nidx);
        double *z = malloc(sizeof(double) * (size_t)(rows * d)), *z2 = malloc(sizeof(double) * (size_t)(rows * d));
        double *g = malloc(sizeof(double) * (size_t)(rows * d)), *gy = malloc(sizeof(double) * (size_t)(rows * d));
        double *dw = malloc(sizeof(double) * (size_t)(m + 1));
        for (int64_t i = 0; i < rows * d; ++i) {
            z[i] = (double)(next() % 1000) / 500.0 - 1.0;
            g[i] = (double)(next() % 1000) / 500.0 - 1.0;
        }
        oracle_sweep(n, m, eptr, eidx, nptr, nidx, w, d, 0.5, 0, z, z2);
        oracle_sweep(n, m, eptr, eidx, nptr, nidx, w, d, 0.5, 1, z, z2);
        oracle_sweep_vjp(n, m, eptr, eidx, nptr, nidx, w, d, 0.5, z, g, gy, dw);
        /* projection and its adjoint onto the coarse level */
        int64_t crows = cn + cm;
        int64_t *rowmap = malloc(sizeof(int64_t) * (size_t)(rows + 1));
        oracle_rowmap(n, m, eptr, eidx, nrep, erep, cn, rowmap);
        double *zc = malloc(sizeof(double) * (size_t)(crows * d + 1)), *gc = malloc(sizeof(double) * (size_t)(crows * d + 1));
        for (int64_t i = 0; i < crows * d; ++i)
            zc[i] = (double)i;
        oracle_project(rows, rowmap, d, zc, z2);
        oracle_project_vjp(rows, crows, rowmap, d, g, gc);
        free(nrep); free(erep); free(x); free(cx); free(fnrep); free(ferep); free(feptr); free(feidx); free(fw);
        free(nptr); free(nidx); free(z); free(z2); free(g); free(gy); free(dw); free(rowmap); free(zc); free(gc);
        free(eptr); free(eidx); free(w);
        /* continue from the coarse level */
        eptr = ceptr;
        eidx = ceidx;
        w = cw;
        n = cn;
        m = cm;
        if (m == 0)
            break;
    }
    free(eptr); free(eidx); free(w);
    return 0;
}

int main(void)
{
    const int64_t shapes[][4] = {{1, 1, 1, 1}, {5, 3, 3, 2}, {40, 25, 6, 3}, {300, 200, 12, 4}, {64, 300, 5, 8},
                                 {1000, 700, 30, 2}};
    for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i)
        if (one_case(shapes[i][0], shapes[i][1], (int)shapes[i][2], shapes[i][3]) != 0) {
            fprintf(stderr, "case %zu failed\n", i);
            return 1;
        }
    printf("oracle sanitizer run ok\n");
    return 0;
}
