/*
 * cr_oracle.c -- plain, slow reference implementation of the persistence
 * diagram of an image's weighted cubical complex over Z/2.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
 * the benchmark's CPU-baseline leg load this library.  The GPU product path
 * never links, calls or executes it, and it shares no code with that path.
 *
 * What it computes (Kaji, Sudo, Ahara, "Cubical Ripser", arXiv:2005.12692):
 *
 *  - The image is a real function on a regular grid (Sec. 2).  A 2D image is a
 *    3D one whose z extent is 1.  C order: x is the fastest axis ("the cell to
 *    the right is (1,0,0)", caption of Fig. 1).
 *  - The weighted cubical complex K(phi) (Sec. 2): its cells are the elementary
 *    cubes of dimension 0..3 spanned by grid vertices.  A cell is addressed here
 *    by Khalimsky coordinates (cz,cy,cx), 0 <= c_a <= 2 n_a - 2, whose odd entries
 *    are the axes it extends along; its dimension is the number of odd entries.
 *    The value (birth time) of a cell is the maximum of the values of the
 *    vertices it contains (the V-construction, Sec. 2).
 *  - A total order on cells refining the filtration: key(c) = (value, dim,
 *    kidx), kidx = (cz*Ky + cy)*Kx + cx with K_a = 2 n_a - 1.  A face never
 *    comes after a coface (smaller or equal value, smaller dimension).  The
 *    paper orders cells of one dimension by (-value, type, z, y, x) for its
 *    cohomology indexing (Sec. 2); pairs with death > birth do not depend on
 *    how ties of value are refined, so this refinement is used on both sides.
 *  - The persistence pairing: the boundary matrix of the filtration, with
 *    columns and rows in key order, is reduced by left-to-right column
 *    additions over Z/2 until every nonzero column has a distinct lowest one
 *    (the standard reduction that the paper's pivots / "upper-triangular form"
 *    refer to, Sec. 2, read in homology).  A column j whose lowest one is in
 *    row i pairs cell i (birth) with cell j (death).  Cells that are neither a
 *    pivot row nor a nonzero column are essential (death = +infinity).
 *    Mode ORACLE_PLAIN reduces all columns in key order.  Mode ORACLE_TWIST
 *    reduces one dimension at a time from the top down and zeroes the column of
 *    every pivot row before its dimension is reduced ("many columns are known
 *    to be reduced to zero without computation", Sec. 2).  Both give the same
 *    pairing because the pairing of a reduced matrix is unique.
 *    Mode ORACLE_COHOMOLOGY is the paper's own formulation (Sec. 2): the
 *    coboundary matrix, columns and rows in reverse key order.  The column of
 *    a cell lists its cofacets; its pivot is the cofacet earliest in key order.
 *    Columns of dimension 0..maxdim are reduced from the latest cell to the
 *    earliest by additions of the columns already reduced.  A nonzero reduced
 *    column pairs its cell (birth) with its pivot (death).  By the duality of
 *    persistent homology and cohomology over a field (from the work the paper
 *    cites for the algorithm), for the same total order the pairs are those of
 *    the homology reduction.  The two share no reduction code.
 *  - Output: the pairs with death > birth (zero-length pairs are dropped) plus
 *    the essential bars, in dimensions 0..maxdim, each with the flat index of
 *    the pixel whose value the birth (death) cell takes: among the vertices of
 *    the cell, the latest in (value, flat index) order.  Rows are in canonical
 *    order: ascending (dim, birth_pixel, death_pixel), an essential bar
 *    (death_pixel = -1) counting as after every finite one.
 *
 * Input conventions: -0.0 is read as +0.0; NaN is an error; +-inf are allowed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

enum { ORACLE_OK = 0, ORACLE_ERR_ARG = 1, ORACLE_ERR_NAN = 2, ORACLE_ERR_TOO_LARGE = 3,
       ORACLE_ERR_NOMEM = 5 };
enum { ORACLE_PLAIN = 0, ORACLE_TWIST = 1, ORACLE_COHOMOLOGY = 2 };

typedef struct {
    int64_t n[3];   /* pixel extents, z y x */
    int64_t K[3];   /* Khalimsky extents 2n-1 */
    int64_t N;      /* number of cells */
    int64_t P;      /* number of pixels */
} grid_t;

typedef struct oracle_result {
    int64_t n_pairs;
    int32_t* dim;
    float* birth;
    float* death;
    int64_t* birth_pixel;
    int64_t* death_pixel;
    /* the full cell pairing, zero-length pairs and essential cells included */
    int64_t n_cell_pairs;
    int64_t* cp_birth;   /* kidx of the birth cell */
    int64_t* cp_death;   /* kidx of the death cell, -1 if essential */
} oracle_result;

/* ---- order-preserving map of an IEEE float onto uint32 ---------------------- */
static uint32_t ord32(float v) {
    uint32_t u;
    memcpy(&u, &v, 4);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

static void coords_of(const grid_t* g, int64_t k, int64_t c[3]) {
    c[2] = k % g->K[2];
    k /= g->K[2];
    c[1] = k % g->K[1];
    c[0] = k / g->K[1];
}

static int64_t kidx_of(const grid_t* g, const int64_t c[3]) {
    return (c[0] * g->K[1] + c[1]) * g->K[2] + c[2];
}

static int dim_of(const int64_t c[3]) {
    return (int)((c[0] & 1) + (c[1] & 1) + (c[2] & 1));
}

/* The vertex of cell c whose value the cell takes: the maximum of its vertex
 * values, ties broken towards the larger flat pixel index. */
static int64_t argmax_vertex(const grid_t* g, const float* img, const int64_t c[3]) {
    int64_t best = -1;
    float bv = 0.0f;
    for (int dz = 0; dz <= (int)(c[0] & 1); ++dz)
        for (int dy = 0; dy <= (int)(c[1] & 1); ++dy)
            for (int dx = 0; dx <= (int)(c[2] & 1); ++dx) {
                int64_t z = c[0] / 2 + dz, y = c[1] / 2 + dy, x = c[2] / 2 + dx;
                int64_t p = (z * g->n[1] + y) * g->n[2] + x;
                float v = img[p];
                if (best < 0 || v > bv || (v == bv && p > best)) {
                    best = p;
                    bv = v;
                }
            }
    return best;
}

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* ---- columns: sorted arrays of row ranks ------------------------------------ */
typedef struct {
    int32_t* v;
    int32_t n;
} col_t;

/* dst = a XOR b (symmetric difference of two ascending lists) */
static int col_xor(const col_t* a, const col_t* b, col_t* dst) {
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)(a->n + b->n + 1));
    if (!out) return -1;
    int32_t i = 0, j = 0, m = 0;
    while (i < a->n && j < b->n) {
        if (a->v[i] < b->v[j]) out[m++] = a->v[i++];
        else if (a->v[i] > b->v[j]) out[m++] = b->v[j++];
        else { ++i; ++j; }
    }
    while (i < a->n) out[m++] = a->v[i++];
    while (j < b->n) out[m++] = b->v[j++];
    dst->v = out;
    dst->n = m;
    return 0;
}

typedef struct {
    int64_t i;  /* sort key for the output rows */
    int64_t bpix, dpix;
    int32_t dim;
    float birth, death;
} row_t;

static int cmp_row(const void* a, const void* b) {
    const row_t* x = (const row_t*)a;
    const row_t* y = (const row_t*)b;
    if (x->dim != y->dim) return x->dim < y->dim ? -1 : 1;
    if (x->bpix != y->bpix) return x->bpix < y->bpix ? -1 : 1;
    uint64_t dx = (uint64_t)x->dpix, dy = (uint64_t)y->dpix; /* -1 sorts last */
    return (dx > dy) - (dx < dy);
}

void oracle_free(oracle_result* r) {
    if (!r) return;
    free(r->dim); free(r->birth); free(r->death);
    free(r->birth_pixel); free(r->death_pixel);
    free(r->cp_birth); free(r->cp_death);
    free(r);
}

int oracle_run(const float* img_in, int ndim, const int64_t* shape, int maxdim, int mode,
               oracle_result** out) {
    if (!out) return ORACLE_ERR_ARG;
    *out = NULL;
    if (!img_in || !shape || ndim < 1 || ndim > 3 || maxdim < 0) return ORACLE_ERR_ARG;
    if (mode != ORACLE_PLAIN && mode != ORACLE_TWIST && mode != ORACLE_COHOMOLOGY) return ORACLE_ERR_ARG;

    grid_t g;
    for (int a = 0; a < 3; ++a) g.n[a] = 1;
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 1) return ORACLE_ERR_ARG;
        g.n[3 - ndim + a] = shape[a];
    }
    g.P = g.n[0] * g.n[1] * g.n[2];
    for (int a = 0; a < 3; ++a) g.K[a] = 2 * g.n[a] - 1;
    g.N = g.K[0] * g.K[1] * g.K[2];
    if (g.N > ((int64_t)1 << 30)) return ORACLE_ERR_TOO_LARGE;
    if (maxdim > ndim - 1) maxdim = ndim - 1;

    /* input: -0.0 read as +0.0, NaN rejected */
    float* img = (float*)malloc(sizeof(float) * (size_t)g.P);
    if (!img) return ORACLE_ERR_NOMEM;
    for (int64_t p = 0; p < g.P; ++p) {
        float v = img_in[p];
        if (v != v) { free(img); return ORACLE_ERR_NAN; }
        img[p] = (v == 0.0f) ? 0.0f : v;
    }

    const int64_t N = g.N;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    float* val = (float*)malloc(sizeof(float) * (size_t)N);
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    if (!keys || !val || !rank) { free(img); free(keys); free(val); free(rank); return ORACLE_ERR_NOMEM; }

    /* cell values (max of vertex values) and keys */
    for (int64_t k = 0; k < N; ++k) {
        int64_t c[3];
        coords_of(&g, k, c);
        float v = img[argmax_vertex(&g, img, c)];
        val[k] = v;
        keys[k] = ((uint64_t)ord32(v) << 32) | ((uint64_t)dim_of(c) << 30) | (uint64_t)k;
    }
    qsort(keys, (size_t)N, sizeof(uint64_t), cmp_u64);
    const uint64_t KMASK = ((uint64_t)1 << 30) - 1;
    for (int64_t i = 0; i < N; ++i) rank[keys[i] & KMASK] = (int32_t)i;
    /* cell (kidx) at each rank */
    int64_t* cell_at = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    int32_t* pivot_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)N); /* row rank -> column rank */
    uint8_t* cleared = (uint8_t*)calloc((size_t)N, 1);
    col_t* R = (col_t*)calloc((size_t)N, sizeof(col_t));
    if (!cell_at || !pivot_col || !cleared || !R) {
        free(img); free(keys); free(val); free(rank); free(cell_at); free(pivot_col); free(cleared); free(R);
        return ORACLE_ERR_NOMEM;
    }
    for (int64_t i = 0; i < N; ++i) {
        cell_at[i] = (int64_t)(keys[i] & KMASK);
        pivot_col[i] = -1;
    }
    free(keys);

    int top = ndim; /* highest cell dimension present in the complex */
    int top_col = maxdim + 1 < top ? maxdim + 1 : top;
    int status = ORACLE_OK;

    /* boundary column of the cell at rank j: ranks of its 2*dim facets, ascending */
    #define LOAD_BOUNDARY(j, colp)                                                   \
        do {                                                                         \
            int64_t c_[3], f_[3];                                                    \
            coords_of(&g, cell_at[(j)], c_);                                         \
            int32_t tmp_[6]; int32_t m_ = 0;                                         \
            for (int a_ = 0; a_ < 3; ++a_) {                                          \
                if (!(c_[a_] & 1)) continue;                                         \
                for (int s_ = -1; s_ <= 1; s_ += 2) {                                \
                    f_[0] = c_[0]; f_[1] = c_[1]; f_[2] = c_[2];                     \
                    f_[a_] += s_;                                                    \
                    tmp_[m_++] = rank[kidx_of(&g, f_)];                              \
                }                                                                    \
            }                                                                        \
            for (int p_ = 1; p_ < m_; ++p_) {                                        \
                int32_t t_ = tmp_[p_]; int q_ = p_ - 1;                              \
                while (q_ >= 0 && tmp_[q_] > t_) { tmp_[q_ + 1] = tmp_[q_]; --q_; }  \
                tmp_[q_ + 1] = t_;                                                   \
            }                                                                        \
            (colp)->v = (int32_t*)malloc(sizeof(int32_t) * 6);                       \
            if (!(colp)->v) { status = ORACLE_ERR_NOMEM; }                           \
            else { memcpy((colp)->v, tmp_, sizeof(int32_t) * (size_t)m_); (colp)->n = m_; } \
        } while (0)

    /* reduce column j against the columns to its left that own its lowest one */
    #define REDUCE(j)                                                                \
        do {                                                                         \
            col_t cur_;                                                              \
            LOAD_BOUNDARY((j), &cur_);                                               \
            if (status != ORACLE_OK) break;                                          \
            while (cur_.n > 0) {                                                     \
                int32_t low_ = cur_.v[cur_.n - 1];                                   \
                int32_t k_ = pivot_col[low_];                                        \
                if (k_ < 0) break;                                                   \
                col_t nxt_;                                                          \
                if (col_xor(&cur_, &R[k_], &nxt_) != 0) { status = ORACLE_ERR_NOMEM; break; } \
                free(cur_.v);                                                        \
                cur_ = nxt_;                                                         \
            }                                                                        \
            if (status != ORACLE_OK) { free(cur_.v); break; }                        \
            if (cur_.n > 0) {                                                        \
                pivot_col[cur_.v[cur_.n - 1]] = (int32_t)(j);                        \
                cleared[cur_.v[cur_.n - 1]] = 1;                                     \
                R[(j)] = cur_;                                                       \
            } else {                                                                 \
                free(cur_.v);                                                        \
            }                                                                        \
        } while (0)

    if (mode == ORACLE_COHOMOLOGY) {
        /* column of the cell at reversed rank q = N-1-rank: the reversed ranks
           of its cofacets, ascending, so that its last entry is the cofacet
           earliest in key order; owner[q'] = the reduced column whose last
           entry is q' */
        int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
        col_t* Q = (col_t*)calloc((size_t)N, sizeof(col_t));
        if (!owner || !Q) status = ORACLE_ERR_NOMEM;
        for (int64_t i = 0; status == ORACLE_OK && i < N; ++i) owner[i] = -1;
        for (int64_t q = 0; q < N && status == ORACLE_OK; ++q) {
            const int64_t j = N - 1 - q;
            int64_t c[3], f[3];
            coords_of(&g, cell_at[j], c);
            const int d = dim_of(c);
            if (d > maxdim || d + 1 > top) continue;
            int32_t tmp[6];
            int m = 0;
            for (int a = 0; a < 3; ++a) {
                if (c[a] & 1) continue;  /* the cell extends along a: no cofacet that way */
                for (int sg = -1; sg <= 1; sg += 2) {
                    f[0] = c[0]; f[1] = c[1]; f[2] = c[2];
                    f[a] += sg;
                    if (f[a] < 0 || f[a] >= g.K[a]) continue;
                    tmp[m++] = (int32_t)(N - 1 - rank[kidx_of(&g, f)]);
                }
            }
            for (int p2 = 1; p2 < m; ++p2) {  /* insertion sort, ascending */
                int32_t t = tmp[p2]; int r2 = p2 - 1;
                while (r2 >= 0 && tmp[r2] > t) { tmp[r2 + 1] = tmp[r2]; --r2; }
                tmp[r2 + 1] = t;
            }
            col_t cur;
            cur.n = m;
            cur.v = (int32_t*)malloc(sizeof(int32_t) * 6);
            if (!cur.v) { status = ORACLE_ERR_NOMEM; break; }
            memcpy(cur.v, tmp, sizeof(int32_t) * (size_t)m);
            while (cur.n > 0) {
                const int32_t low = cur.v[cur.n - 1];
                const int32_t k = owner[low];
                if (k < 0) break;
                col_t nxt;
                if (col_xor(&cur, &Q[k], &nxt) != 0) { status = ORACLE_ERR_NOMEM; break; }
                free(cur.v);
                cur = nxt;
            }
            if (status != ORACLE_OK) { free(cur.v); break; }
            if (cur.n > 0) {
                const int32_t low = cur.v[cur.n - 1];
                owner[low] = (int32_t)q;
                Q[q] = cur;
                pivot_col[j] = (int32_t)(N - 1 - low);  /* birth rank j, death rank of the pivot */
            } else {
                free(cur.v);
            }
        }
        if (Q) for (int64_t i = 0; i < N; ++i) free(Q[i].v);
        free(Q);
        free(owner);
    } else if (mode == ORACLE_PLAIN) {
        for (int64_t j = 0; j < N && status == ORACLE_OK; ++j) {
            int64_t c[3];
            coords_of(&g, cell_at[j], c);
            int d = dim_of(c);
            if (d == 0 || d > top_col) continue;
            REDUCE(j);
        }
    } else {
        for (int d = top_col; d >= 1 && status == ORACLE_OK; --d) {
            for (int64_t j = 0; j < N && status == ORACLE_OK; ++j) {
                int64_t c[3];
                coords_of(&g, cell_at[j], c);
                if (dim_of(c) != d) continue;
                if (cleared[j]) continue; /* a pivot row of dimension d+1: its column is zero */
                REDUCE(j);
            }
        }
    }
    #undef REDUCE
    #undef LOAD_BOUNDARY

    oracle_result* res = NULL;
    row_t* rows = NULL;
    if (status == ORACLE_OK) {
        /* inverse of pivot_col: column rank -> row rank */
        int32_t* low_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
        res = (oracle_result*)calloc(1, sizeof(oracle_result));
        if (!low_of || !res) status = ORACLE_ERR_NOMEM;
        if (status == ORACLE_OK) {
            for (int64_t i = 0; i < N; ++i) low_of[i] = -1;
            for (int64_t i = 0; i < N; ++i)
                if (pivot_col[i] >= 0) low_of[pivot_col[i]] = (int32_t)i;
            /* full cell pairing in dimensions 0..maxdim */
            int64_t ncp = 0, nrows = 0;
            for (int64_t i = 0; i < N; ++i) {
                int64_t c[3];
                coords_of(&g, cell_at[i], c);
                int d = dim_of(c);
                if (d > maxdim) continue;
                if (pivot_col[i] >= 0) ++ncp;                 /* birth of a finite pair */
                else if (low_of[i] < 0) ++ncp;                /* essential */
            }
            res->cp_birth = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncp + 1));
            res->cp_death = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncp + 1));
            rows = (row_t*)malloc(sizeof(row_t) * (size_t)(ncp + 1));
            if (!res->cp_birth || !res->cp_death || !rows) status = ORACLE_ERR_NOMEM;
            if (status == ORACLE_OK) {
                int64_t m = 0;
                for (int64_t i = 0; i < N; ++i) {
                    int64_t c[3];
                    coords_of(&g, cell_at[i], c);
                    int d = dim_of(c);
                    if (d > maxdim) continue;
                    int64_t j = -1;
                    if (pivot_col[i] >= 0) j = pivot_col[i];
                    else if (low_of[i] >= 0) continue; /* a death cell */
                    res->cp_birth[m] = cell_at[i];
                    res->cp_death[m] = j >= 0 ? cell_at[j] : -1;
                    ++m;
                    float b = val[cell_at[i]];
                    float dv = j >= 0 ? val[cell_at[j]] : INFINITY;
                    if (j >= 0 && !(dv > b)) continue; /* zero-length pair */
                    row_t r;
                    r.dim = d;
                    r.birth = b;
                    r.death = dv;
                    r.bpix = argmax_vertex(&g, img, c);
                    if (j >= 0) {
                        int64_t cd[3];
                        coords_of(&g, cell_at[j], cd);
                        r.dpix = argmax_vertex(&g, img, cd);
                    } else {
                        r.dpix = -1;
                    }
                    r.i = nrows;
                    rows[nrows++] = r;
                }
                res->n_cell_pairs = m;
                qsort(rows, (size_t)nrows, sizeof(row_t), cmp_row);
                res->n_pairs = nrows;
                size_t nn = (size_t)(nrows + 1);
                res->dim = (int32_t*)malloc(sizeof(int32_t) * nn);
                res->birth = (float*)malloc(sizeof(float) * nn);
                res->death = (float*)malloc(sizeof(float) * nn);
                res->birth_pixel = (int64_t*)malloc(sizeof(int64_t) * nn);
                res->death_pixel = (int64_t*)malloc(sizeof(int64_t) * nn);
                if (!res->dim || !res->birth || !res->death || !res->birth_pixel || !res->death_pixel)
                    status = ORACLE_ERR_NOMEM;
                else
                    for (int64_t i = 0; i < nrows; ++i) {
                        res->dim[i] = rows[i].dim;
                        res->birth[i] = rows[i].birth;
                        res->death[i] = rows[i].death;
                        res->birth_pixel[i] = rows[i].bpix;
                        res->death_pixel[i] = rows[i].dpix;
                    }
            }
        }
        free(low_of);
    }
    free(rows);
    for (int64_t i = 0; i < N; ++i) free(R[i].v);
    free(R); free(cleared); free(pivot_col); free(cell_at); free(rank); free(val); free(img);
    if (status != ORACLE_OK) { oracle_free(res); return status; }
    *out = res;
    return ORACLE_OK;
}

int64_t oracle_n_pairs(const oracle_result* r) { return r ? r->n_pairs : 0; }
int64_t oracle_n_cell_pairs(const oracle_result* r) { return r ? r->n_cell_pairs : 0; }

void oracle_get_pairs(const oracle_result* r, int32_t* dim, float* birth, float* death,
                      int64_t* birth_pixel, int64_t* death_pixel) {
    size_t n = (size_t)r->n_pairs;
    if (n == 0) return;  /* the arrays may be NULL then (memcpy from NULL is undefined) */
    if (dim) memcpy(dim, r->dim, n * sizeof(int32_t));
    if (birth) memcpy(birth, r->birth, n * sizeof(float));
    if (death) memcpy(death, r->death, n * sizeof(float));
    if (birth_pixel) memcpy(birth_pixel, r->birth_pixel, n * sizeof(int64_t));
    if (death_pixel) memcpy(death_pixel, r->death_pixel, n * sizeof(int64_t));
}

void oracle_get_cell_pairs(const oracle_result* r, int64_t* birth_kidx, int64_t* death_kidx) {
    size_t n = (size_t)r->n_cell_pairs;
    if (n == 0) return;  /* the degree-0 union-find keeps no cell pairing: NULL arrays */
    if (birth_kidx) memcpy(birth_kidx, r->cp_birth, n * sizeof(int64_t));
    if (death_kidx) memcpy(death_kidx, r->cp_death, n * sizeof(int64_t));
}

/* ---- degree 0 by union-find (Sec. 2, Fig. 2) ---------------------------------
 * The paper's own description of the 0-th persistence: visit the 1-cells in
 * increasing order of the filtration; an edge joining two components kills the
 * component born later (the elder rule), and the older component survives.
 * Connectivity is 4-neighbour in 2D and 6-neighbour in 3D.  "Later" is the
 * total order of keys used above, so this gives the same pairing as the
 * reduction in degree 0; it needs only O(#edges) memory, so it runs on inputs
 * far larger than the full reduction can. */
static int64_t uf_find(int64_t* parent, int64_t x) {
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) { int64_t nx = parent[x]; parent[x] = r; x = nx; }
    return r;
}

int oracle_h0_run(const float* img_in, int ndim, const int64_t* shape, oracle_result** out) {
    if (!out) return ORACLE_ERR_ARG;
    *out = NULL;
    if (!img_in || !shape || ndim < 1 || ndim > 3) return ORACLE_ERR_ARG;
    grid_t g;
    for (int a = 0; a < 3; ++a) g.n[a] = 1;
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 1) return ORACLE_ERR_ARG;
        g.n[3 - ndim + a] = shape[a];
    }
    g.P = g.n[0] * g.n[1] * g.n[2];
    for (int a = 0; a < 3; ++a) g.K[a] = 2 * g.n[a] - 1;
    g.N = g.K[0] * g.K[1] * g.K[2];
    if (g.N > ((int64_t)1 << 30)) return ORACLE_ERR_TOO_LARGE;

    float* img = (float*)malloc(sizeof(float) * (size_t)g.P);
    if (!img) return ORACLE_ERR_NOMEM;
    for (int64_t p = 0; p < g.P; ++p) {
        float v = img_in[p];
        if (v != v) { free(img); return ORACLE_ERR_NAN; }
        img[p] = (v == 0.0f) ? 0.0f : v;
    }
    /* all edges: one per (pixel, axis) with a neighbour along +axis */
    int64_t ne = 0;
    for (int a = 0; a < 3; ++a) ne += (g.n[a] - 1) * (g.P / g.n[a]);
    uint64_t* ekeys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(ne + 1));
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)g.P);
    if (!ekeys || !parent) { free(img); free(ekeys); free(parent); return ORACLE_ERR_NOMEM; }
    int64_t m = 0;
    for (int64_t z = 0; z < g.n[0]; ++z)
        for (int64_t y = 0; y < g.n[1]; ++y)
            for (int64_t x = 0; x < g.n[2]; ++x)
                for (int a = 0; a < 3; ++a) {
                    int64_t c[3] = {2 * z, 2 * y, 2 * x};
                    if (c[a] / 2 + 1 >= g.n[a]) continue;
                    c[a] += 1;
                    float v = img[argmax_vertex(&g, img, c)];
                    ekeys[m++] = ((uint64_t)ord32(v) << 32) | ((uint64_t)1 << 30) |
                                 (uint64_t)kidx_of(&g, c);
                }
    qsort(ekeys, (size_t)m, sizeof(uint64_t), cmp_u64);
    for (int64_t p = 0; p < g.P; ++p) parent[p] = p;

    /* the key of a vertex, for the elder comparison */
    #define VKEY(p) (((uint64_t)ord32(img[(p)]) << 32) |                                 \
                     (uint64_t)kidx_of(&g, (int64_t[3]){2 * ((p) / (g.n[1] * g.n[2])),      \
                                                       2 * (((p) / g.n[2]) % g.n[1]),       \
                                                       2 * ((p) % g.n[2])}))
    row_t* rows = (row_t*)malloc(sizeof(row_t) * (size_t)(g.P + 1));
    if (!rows) { free(img); free(ekeys); free(parent); return ORACLE_ERR_NOMEM; }
    int64_t nrows = 0;
    const uint64_t KMASK = ((uint64_t)1 << 30) - 1;
    for (int64_t i = 0; i < m; ++i) {
        int64_t c[3], u[3];
        coords_of(&g, (int64_t)(ekeys[i] & KMASK), c);
        int a = (c[0] & 1) ? 0 : (c[1] & 1) ? 1 : 2;
        u[0] = c[0]; u[1] = c[1]; u[2] = c[2];
        u[a] -= 1;
        int64_t p = (u[0] / 2 * g.n[1] + u[1] / 2) * g.n[2] + u[2] / 2;
        u[a] += 2;
        int64_t q = (u[0] / 2 * g.n[1] + u[1] / 2) * g.n[2] + u[2] / 2;
        int64_t rp = uf_find(parent, p), rq = uf_find(parent, q);
        if (rp == rq) continue;
        uint64_t kp = VKEY(rp), kq = VKEY(rq);
        int64_t young = kp > kq ? rp : rq, old = kp > kq ? rq : rp;
        float dv = img[argmax_vertex(&g, img, c)];
        if (dv > img[young]) {
            row_t r;
            r.dim = 0;
            r.birth = img[young];
            r.death = dv;
            r.bpix = young;
            r.dpix = argmax_vertex(&g, img, c);
            r.i = nrows;
            rows[nrows++] = r;
        }
        parent[young] = old;
    }
    #undef VKEY
    /* the essential bar: the root of the (single) component */
    int64_t root = uf_find(parent, 0);
    {
        row_t r;
        r.dim = 0; r.birth = img[root]; r.death = INFINITY; r.bpix = root; r.dpix = -1; r.i = nrows;
        rows[nrows++] = r;
    }
    qsort(rows, (size_t)nrows, sizeof(row_t), cmp_row);
    oracle_result* res = (oracle_result*)calloc(1, sizeof(oracle_result));
    int status = res ? ORACLE_OK : ORACLE_ERR_NOMEM;
    if (res) {
        size_t nn = (size_t)nrows + 1;
        res->n_pairs = nrows;
        res->dim = (int32_t*)malloc(sizeof(int32_t) * nn);
        res->birth = (float*)malloc(sizeof(float) * nn);
        res->death = (float*)malloc(sizeof(float) * nn);
        res->birth_pixel = (int64_t*)malloc(sizeof(int64_t) * nn);
        res->death_pixel = (int64_t*)malloc(sizeof(int64_t) * nn);
        if (!res->dim || !res->birth || !res->death || !res->birth_pixel || !res->death_pixel)
            status = ORACLE_ERR_NOMEM;
        else
            for (int64_t i = 0; i < nrows; ++i) {
                res->dim[i] = 0;
                res->birth[i] = rows[i].birth;
                res->death[i] = rows[i].death;
                res->birth_pixel[i] = rows[i].bpix;
                res->death_pixel[i] = rows[i].dpix;
            }
    }
    free(rows); free(ekeys); free(parent); free(img);
    if (status != ORACLE_OK) { oracle_free(res); return status; }
    *out = res;
    return ORACLE_OK;
}
