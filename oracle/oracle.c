/*
 * CPU oracle for the local sparse product C = A (x) B over a semiring.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library. The GPU library
 * shares no code, header, table or helper with it.
 *
 * What it computes (paper, Section 1 and Eq. 1): for every output position
 *     C(i, j) = (+)_{k : A(i,k) and B(k,j) stored} A(i,k) (x) B(k,j),
 * keeping every produced position (a structural product: a position whose
 * accumulated value equals the additive identity is still stored).
 *
 * How: the classical column-by-column algorithm of Gustavson (Section 1,
 * Section 3.3 and 4.1) with a dense sparse accumulator (SPA). For each stored
 * column j of B in ascending order, for each (k, b) of B(:, j) in ascending k,
 * for each (i, a) of A(:, k) in ascending i, the product a (x) b is added
 * into w[i]; a mark array tells whether w[i] was already started for this
 * column, and a list records the touched rows. The list is then sorted and
 * emitted. Values are therefore accumulated in ascending k.
 *
 * The row-major case C = A B with A, B in CSR/DCSR runs the same routine on
 * the transposes (C^T = B^T A^T, and CSR of X is CSC of X^T) while keeping
 * the multiplication operand order A(i,k) (x) B(k,j).
 *
 * Doubly compressed operands (DCSC, Section 2.3): column k of the gathered
 * operand is located by binary search of k in its JC array; a missing k is an
 * empty column and contributes no work (the Isect observation of Section 2.4).
 *
 * Semirings: (+,*) on double and on float (each accumulates in its own type),
 * (min,+) on int32 with INT32_MAX as the additive identity (+infinity) and
 * saturating addition as the multiply, and (or,and) on a boolean pattern.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_PLUS_TIMES_F64 = 0,
    ORC_PLUS_TIMES_F32 = 1,
    ORC_MIN_PLUS_I32 = 2,
    ORC_OR_AND_BOOL = 3,
};

typedef struct {
    int64_t nvec;        /* number of stored vectors                          */
    const int32_t *vid;  /* major id of each stored vector, or NULL (id = t)  */
    const int64_t *ptr;  /* nvec + 1 offsets                                  */
    const int32_t *idx;  /* minor ids, ascending inside each vector           */
    const void *val;     /* values, or NULL for a boolean pattern             */
} orc_vecs;

typedef struct {
    int64_t nvec, nnz, flops;
    int32_t *vid;        /* major ids of the non-empty output vectors */
    int64_t *ptr;        /* nvec + 1 */
    int32_t *idx;
    void *val;           /* NULL for boolean */
} orc_result;

static int64_t orc_sat_add(int32_t a, int32_t b)
{
    if (a == INT32_MAX || b == INT32_MAX)
        return INT32_MAX;
    int64_t s = (int64_t)a + (int64_t)b;
    if (s > INT32_MAX)
        return INT32_MAX;
    if (s < INT32_MIN)
        return INT32_MIN;
    return s;
}

static size_t orc_vsize(int sr)
{
    switch (sr) {
    case ORC_PLUS_TIMES_F64: return 8;
    case ORC_PLUS_TIMES_F32: return 4;
    case ORC_MIN_PLUS_I32: return 4;
    default: return 0;
    }
}

static int orc_cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* locate stored vector with major id k; -1 if absent */
static int64_t orc_find(const orc_vecs *m, int64_t k)
{
    if (m->vid == NULL)
        return (k >= 0 && k < m->nvec) ? k : -1;
    int64_t lo = 0, hi = m->nvec;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (m->vid[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < m->nvec && m->vid[lo] == k) ? lo : -1;
}

static int orc_grow(orc_result *r, int64_t need, int64_t *cap, size_t vs)
{
    if (need <= *cap)
        return 0;
    int64_t nc = *cap ? *cap : 1024;
    while (nc < need)
        nc *= 2;
    int32_t *ni = (int32_t *)realloc(r->idx, (size_t)nc * sizeof(int32_t));
    if (!ni)
        return -1;
    r->idx = ni;
    if (vs) {
        void *nv = realloc(r->val, (size_t)nc * vs);
        if (!nv)
            return -1;
        r->val = nv;
    }
    *cap = nc;
    return 0;
}

/*
 * Column-wise product. G holds the gathered columns (A of C = A B), S the
 * streamed columns (B). m = number of rows of G (= of C). gfirst = 1 means the
 * product is g (x) s, else s (x) g. S's vectors define the output vectors.
 * Returns 0, or -1 on allocation failure / bad semiring, -2 on an id out of
 * range.
 */
int orc_colwise(int sr, int gfirst, int64_t m, const orc_vecs *G, const orc_vecs *S,
                orc_result *out)
{
    size_t vs = orc_vsize(sr);
    if (sr < 0 || sr > 3)
        return -1;
    memset(out, 0, sizeof(*out));
    int64_t *mark = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int32_t *list = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    double *wd = NULL;
    float *wf = NULL;
    int32_t *wi = NULL;
    if (sr == ORC_PLUS_TIMES_F64) wd = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (sr == ORC_PLUS_TIMES_F32) wf = (float *)malloc((size_t)(m > 0 ? m : 1) * sizeof(float));
    if (sr == ORC_MIN_PLUS_I32) wi = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    out->vid = (int32_t *)malloc((size_t)(S->nvec > 0 ? S->nvec : 1) * sizeof(int32_t));
    out->ptr = (int64_t *)malloc((size_t)(S->nvec + 1) * sizeof(int64_t));
    int rc = 0;
    if (!mark || !list || !out->vid || !out->ptr || (vs && !wd && !wf && !wi)) {
        rc = -1;
        goto done;
    }
    for (int64_t i = 0; i < m; ++i)
        mark[i] = -1;
    int64_t cap = 0, nnz = 0, flops = 0, nout = 0;
    out->ptr[0] = 0;
    for (int64_t t = 0; t < S->nvec; ++t) {
        int64_t j = S->vid ? S->vid[t] : t;
        int64_t nl = 0;
        for (int64_t e = S->ptr[t]; e < S->ptr[t + 1]; ++e) {
            int64_t k = S->idx[e];
            int64_t gt = orc_find(G, k);
            if (gt < 0)
                continue;
            flops += G->ptr[gt + 1] - G->ptr[gt];
            for (int64_t q = G->ptr[gt]; q < G->ptr[gt + 1]; ++q) {
                int64_t i = G->idx[q];
                if (i < 0 || i >= m) {
                    rc = -2;
                    goto done;
                }
                int first = mark[i] != j;
                if (first) {
                    mark[i] = j;
                    list[nl++] = (int32_t)i;
                }
                switch (sr) {
                case ORC_PLUS_TIMES_F64: {
                    double g = ((const double *)G->val)[q], s = ((const double *)S->val)[e];
                    double p = gfirst ? g * s : s * g;
                    wd[i] = first ? p : wd[i] + p;
                    break;
                }
                case ORC_PLUS_TIMES_F32: {
                    float g = ((const float *)G->val)[q], s = ((const float *)S->val)[e];
                    float p = gfirst ? g * s : s * g;
                    wf[i] = first ? p : wf[i] + p;
                    break;
                }
                case ORC_MIN_PLUS_I32: {
                    int32_t g = ((const int32_t *)G->val)[q], s = ((const int32_t *)S->val)[e];
                    int32_t p = (int32_t)(gfirst ? orc_sat_add(g, s) : orc_sat_add(s, g));
                    wi[i] = first ? p : (p < wi[i] ? p : wi[i]);
                    break;
                }
                default:
                    break;
                }
            }
        }
        if (nl == 0)
            continue;
        qsort(list, (size_t)nl, sizeof(int32_t), orc_cmp_i32);
        if (orc_grow(out, nnz + nl, &cap, vs)) {
            rc = -1;
            goto done;
        }
        for (int64_t q = 0; q < nl; ++q) {
            int32_t i = list[q];
            out->idx[nnz + q] = i;
            if (sr == ORC_PLUS_TIMES_F64) ((double *)out->val)[nnz + q] = wd[i];
            if (sr == ORC_PLUS_TIMES_F32) ((float *)out->val)[nnz + q] = wf[i];
            if (sr == ORC_MIN_PLUS_I32) ((int32_t *)out->val)[nnz + q] = wi[i];
        }
        nnz += nl;
        out->vid[nout] = (int32_t)j;
        out->ptr[++nout] = nnz;
    }
    out->nvec = nout;
    out->nnz = nnz;
    out->flops = flops;
done:
    free(mark);
    free(list);
    free(wd);
    free(wf);
    free(wi);
    return rc;
}

void orc_free(orc_result *r)
{
    free(r->vid);
    free(r->ptr);
    free(r->idx);
    free(r->val);
    memset(r, 0, sizeof(*r));
}
