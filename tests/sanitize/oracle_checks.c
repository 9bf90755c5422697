/*
 * Driver of the oracle's sanitizer build (test infrastructure).
 *
 * Compiled together with oracle/cr_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it runs the oracle on the worked examples of the
 * paper (the TTK image of Remark 3.2, an image matching the caption of
 * Fig. 2, the 3D void) and on many small random grids in 1D, 2D and 3D, in both
 * reduction modes and through the degree-0 union-find, and checks what fixes
 * the result without the oracle's own arithmetic: the printed bars of the
 * worked examples, plain == twist, degree 0 of the reduction == the union-find,
 * exactly one essential bar (in degree 0, at the global minimum),
 * birth < death, and birth/death equal to the pixel values they point at.
 * Any sanitizer report aborts the process; the exit status is the number of
 * failed checks.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_result oracle_result;
int oracle_run(const float* img, int ndim, const int64_t* shape, int maxdim, int mode, oracle_result** out);
int oracle_h0_run(const float* img, int ndim, const int64_t* shape, oracle_result** out);
int64_t oracle_n_pairs(const oracle_result* r);
int64_t oracle_n_cell_pairs(const oracle_result* r);
void oracle_get_pairs(const oracle_result* r, int32_t* dim, float* birth, float* death, int64_t* bp, int64_t* dp);
void oracle_get_cell_pairs(const oracle_result* r, int64_t* b, int64_t* d);
void oracle_free(oracle_result* r);

static int failures = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);                     \
      fprintf(stderr, "\n");                            \
      ++failures;                                       \
    }                                                   \
  } while (0)

typedef struct {
  int64_t n;
  int32_t* dim;
  float *birth, *death;
  int64_t *bp, *dp;
} rows_t;

static rows_t fetch(oracle_result* r) {
  rows_t x;
  x.n = oracle_n_pairs(r);
  size_t m = (size_t)(x.n ? x.n : 1);
  x.dim = malloc(m * sizeof(int32_t));
  x.birth = malloc(m * sizeof(float));
  x.death = malloc(m * sizeof(float));
  x.bp = malloc(m * sizeof(int64_t));
  x.dp = malloc(m * sizeof(int64_t));
  oracle_get_pairs(r, x.dim, x.birth, x.death, x.bp, x.dp);
  /* the full cell pairing is exported too: fetch it so its copy is exercised */
  int64_t nc = oracle_n_cell_pairs(r);
  int64_t* cb = malloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
  int64_t* cd = malloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
  oracle_get_cell_pairs(r, cb, cd);
  free(cb);
  free(cd);
  return x;
}
static void rows_free(rows_t* x) {
  free(x->dim); free(x->birth); free(x->death); free(x->bp); free(x->dp);
}

static rows_t run(const float* img, int ndim, const int64_t* shape, int maxdim, int mode) {
  oracle_result* r = NULL;
  int rc = oracle_run(img, ndim, shape, maxdim, mode, &r);
  CHECK(rc == 0 && r, "oracle_run returned %d", rc);
  rows_t x = fetch(r);
  oracle_free(r);
  return x;
}

static int same(const rows_t* a, const rows_t* b, int dim_only0) {
  int64_t na = 0, nb = 0;
  for (int64_t i = 0; i < a->n; ++i) na += !dim_only0 || a->dim[i] == 0;
  for (int64_t i = 0; i < b->n; ++i) nb += !dim_only0 || b->dim[i] == 0;
  if (na != nb) return 0;
  for (int64_t i = 0, j = 0; i < a->n && j < b->n; ++i, ++j) {
    while (dim_only0 && i < a->n && a->dim[i] != 0) ++i;
    while (dim_only0 && j < b->n && b->dim[j] != 0) ++j;
    if (i >= a->n || j >= b->n) break;
    if (a->dim[i] != b->dim[j] || memcmp(&a->birth[i], &b->birth[j], 4) || memcmp(&a->death[i], &b->death[j], 4) ||
        a->bp[i] != b->bp[j] || a->dp[i] != b->dp[j])
      return 0;
  }
  return 1;
}

static void invariants(const rows_t* x, const float* img, int64_t P, const char* what) {
  int ess = 0;
  float mn = INFINITY;
  for (int64_t p = 0; p < P; ++p) mn = img[p] < mn ? img[p] : mn;
  for (int64_t i = 0; i < x->n; ++i) {
    CHECK(x->bp[i] >= 0 && x->bp[i] < P, "%s: birth pixel out of range", what);
    CHECK(memcmp(&x->birth[i], &img[x->bp[i]], 4) == 0 || (x->birth[i] == 0.0f && img[x->bp[i]] == 0.0f),
          "%s: birth is not the value at its pixel", what);
    if (x->dp[i] < 0) {
      ++ess;
      CHECK(x->dim[i] == 0 && x->birth[i] == mn && isinf(x->death[i]), "%s: bad essential bar", what);
    } else {
      CHECK(x->dp[i] < P, "%s: death pixel out of range", what);
      CHECK(x->birth[i] < x->death[i], "%s: birth >= death", what);
      CHECK(memcmp(&x->death[i], &img[x->dp[i]], 4) == 0 || (x->death[i] == 0.0f && img[x->dp[i]] == 0.0f),
            "%s: death is not the value at its pixel", what);
    }
  }
  CHECK(ess == 1, "%s: %d essential bars", what, ess);
}

static uint64_t rng = 88172645463325252ull;
static uint32_t next(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (uint32_t)(rng >> 11);
}

int main(void) {
  /* Remark 3.2: the TTK image, H0 {[0, inf)}, H1 {[0, 9)} */
  {
    const float img[9] = {0, 0, 0, 0, 9, 0, 0, 0, 0};
    const int64_t sh[2] = {3, 3};
    rows_t x = run(img, 2, sh, 1, 1);
    CHECK(x.n == 2, "ttk: %lld rows", (long long)x.n);
    if (x.n == 2) {
      CHECK(x.dim[0] == 0 && x.birth[0] == 0 && isinf(x.death[0]), "ttk: H0 bar");
      CHECK(x.dim[1] == 1 && x.birth[1] == 0 && x.death[1] == 9 && x.dp[1] == 4, "ttk: H1 bar");
    }
    rows_free(&x);
  }
  /* the caption of Fig. 2: H0 {[-2, inf), [-1, 1), [-1, 2)}, empty H1 */
  {
    const float img[9] = {-1, 1, -2, 3, 3, 2, 3, 3, -1};
    const int64_t sh[2] = {3, 3};
    rows_t x = run(img, 2, sh, 1, 1);
    int h0 = 0, one = 0, two = 0;
    for (int64_t i = 0; i < x.n; ++i) {
      CHECK(x.dim[i] == 0, "fig2: a bar of degree %d", x.dim[i]);
      h0 += x.dim[i] == 0;
      one += x.birth[i] == -1 && x.death[i] == 1;
      two += x.birth[i] == -1 && x.death[i] == 2;
    }
    CHECK(h0 == 3 && one == 1 && two == 1, "fig2: %d bars", h0);
    rows_free(&x);
  }
  /* a 3x3x3 void: H0 {[0, inf)}, H2 {[0, 9)} */
  {
    float img[27] = {0};
    img[13] = 9;
    const int64_t sh[3] = {3, 3, 3};
    rows_t x = run(img, 3, sh, 2, 1);
    CHECK(x.n == 2 && x.dim[1] == 2 && x.death[1] == 9, "void: %lld rows", (long long)x.n);
    rows_free(&x);
  }
  /* random grids: plain == twist, degree 0 == the union-find, invariants */
  for (int t = 0; t < 300; ++t) {
    const int ndim = 1 + t % 3;
    int64_t sh[3] = {1, 1, 1};
    int64_t P = 1;
    for (int a = 0; a < ndim; ++a) {
      sh[a] = 1 + next() % (ndim == 3 ? 5 : (ndim == 2 ? 9 : 40));
      P *= sh[a];
    }
    const uint32_t levels = t % 4 == 0 ? 3 : 1000;
    float* img = malloc((size_t)P * sizeof(float));
    for (int64_t p = 0; p < P; ++p) img[p] = (float)(next() % levels) - (float)(levels / 2);
    if (t % 7 == 3) img[next() % P] = INFINITY;
    if (t % 11 == 5) img[next() % P] = -0.0f;
    char what[64];
    snprintf(what, sizeof what, "case %d (ndim %d)", t, ndim);
    rows_t a = run(img, ndim, sh, ndim - 1, 0);
    rows_t b = run(img, ndim, sh, ndim - 1, 1);
    CHECK(same(&a, &b, 0), "%s: plain and twist differ", what);
    invariants(&b, img, P, what);
    oracle_result* r = NULL;
    int rc = oracle_h0_run(img, ndim, sh, &r);
    CHECK(rc == 0, "%s: oracle_h0_run returned %d", what, rc);
    rows_t c = fetch(r);
    oracle_free(r);
    CHECK(same(&b, &c, 1), "%s: degree 0 differs from the union-find", what);
    rows_free(&a);
    rows_free(&b);
    rows_free(&c);
    free(img);
  }
  /* argument errors and NaN */
  {
    const float img[4] = {0, NAN, 1, 2};
    const int64_t sh[2] = {2, 2};
    oracle_result* r = NULL;
    CHECK(oracle_run(img, 2, sh, 1, 1, &r) == 2 && r == NULL, "NaN not reported");
    CHECK(oracle_run(NULL, 2, sh, 1, 1, &r) == 1, "NULL image accepted");
    CHECK(oracle_run(img, 4, sh, 1, 1, &r) == 1, "ndim 4 accepted");
  }
  printf("oracle sanitizer checks: %d failures\n", failures);
  return failures;
}
