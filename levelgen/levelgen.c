/*
 * levelgen.c - seeded synthetic level-structured symmetric matrices.
 *
 * Stand-in for the hierarchical CI Hamiltonians of the paper (Sec. I, Sec. VI.A,
 * Table 1): the basis is split into levels l = 0..L-1 (the analogue of the N_max
 * shells), the leading levels form the small configuration space, and matrix
 * elements couple states of the same level or of adjacent levels only.
 *
 * Recipe (one fixed reading, used by every consumer of these inputs):
 *   - diagonal   H_rr = 10*l(r) + U(-1,1)
 *   - each row r of level l draws floor(d/2) column indices c uniformly from the
 *     window [off[max(0,l-1)], off[min(L,l+2)]); a draw with c == r is dropped;
 *     every drawn pair {r,c} gets one value v ~ N(0, 0.5^2) stored at (r,c) and
 *     (c,r); when an unordered pair is drawn more than once, the draw with the
 *     smallest (drawing row, draw index) wins.
 *   - every value (diagonal too) is rounded to float32, so float32 storage of
 *     the matrix is exact.
 *   - random numbers come from a counter-based generator: the splitmix64
 *     finalizer chained over (seed, stream, row, draw).  Each draw is a pure
 *     function of its counters, so generation is parallel and reproducible.
 *
 * Output: the upper triangle (diagonal included) as CSR with int64 row
 * pointers, int32 column indices sorted ascending within each row, and float32
 * values.  This file holds no arithmetic of the eigensolver.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* stream ids */
enum { S_COL = 1, S_VAL_A = 2, S_VAL_B = 3, S_DIAG = 4 };

static inline uint64_t ctr(uint64_t seed, uint64_t stream, uint64_t row, uint64_t draw) {
  return mix64(mix64(mix64(seed ^ (stream << 56)) ^ row) ^ draw);
}

static inline double u01(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

static inline float gauss_half(uint64_t seed, uint64_t row, uint64_t t) {
  /* Box-Muller, sigma = 0.5 */
  double u1 = ((double)(ctr(seed, S_VAL_A, row, t) >> 11) + 1.0) * 0x1.0p-53; /* (0,1] */
  double u2 = u01(ctr(seed, S_VAL_B, row, t));
  double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
  return (float)(0.5 * g);
}

typedef struct {
  int32_t j;   /* column (the larger index of the pair) */
  float v;     /* value */
  uint64_t key;/* drawing row * 1024 + draw index: the smallest key wins */
} entry_t;

static int cmp_entry(const void* a, const void* b) {
  const entry_t* x = (const entry_t*)a;
  const entry_t* y = (const entry_t*)b;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return 0;
}

static inline int level_of(const int64_t* off, int L, int64_t r) {
  int lo = 0, hi = L - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* Draw t of row r: writes the column into *c; returns 0 if the draw is dropped. */
static inline int draw_col(uint64_t seed, const int64_t* off, int L, int64_t r, int l,
                           int t, int64_t* c) {
  int64_t lo = off[l > 0 ? l - 1 : 0];
  int64_t hi = off[l + 2 < L ? l + 2 : L];
  uint64_t w = (uint64_t)(hi - lo);
  uint64_t z = ctr(seed, S_COL, (uint64_t)r, (uint64_t)t);
  int64_t cc = lo + (int64_t)(((z >> 32) * w) >> 32);
  *c = cc;
  return cc != r;
}

/*
 * Generate.  level_sizes[L], d = target mean full-row degree, seed.
 * On success returns 0 and sets *n_out, *nnz_out and malloc'ed arrays
 * (free them with levelgen_free).  Returns -1 on bad arguments, -2 on
 * allocation failure.
 */
int levelgen_generate(const int64_t* level_sizes, int L, int d, uint64_t seed,
                      int64_t* n_out, int64_t* nnz_out,
                      int64_t** row_ptr_out, int32_t** col_out, float** val_out) {
  if (L < 1 || L > 64 || d < 0 || d / 2 > 1000) return -1;
  int64_t off[65];
  off[0] = 0;
  for (int l = 0; l < L; ++l) {
    if (level_sizes[l] <= 0) return -1;
    off[l + 1] = off[l] + level_sizes[l];
  }
  const int64_t n = off[L];
  if (n >= (int64_t)1 << 31) return -1;
  const int h = d / 2;

  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;

  /* pass 1: count the strict-upper entries owned by each row (owner = smaller index) */
#pragma omp parallel for schedule(static, 4096)
  for (int64_t r = 0; r < n; ++r) {
    int l = level_of(off, L, r);
    for (int t = 0; t < h; ++t) {
      int64_t c;
      if (!draw_col(seed, off, L, r, l, t, &c)) continue;
      int64_t owner = c < r ? c : r;
#pragma omp atomic
      cnt[owner + 1] += 1;
    }
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  const int64_t total = cnt[n];

  entry_t* ent = (entry_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(entry_t));
  int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!ent || !fill) { free(cnt); free(ent); free(fill); return -2; }
  memcpy(fill, cnt, (size_t)n * sizeof(int64_t));

  /* pass 2: scatter every draw into its owner's segment */
#pragma omp parallel for schedule(static, 4096)
  for (int64_t r = 0; r < n; ++r) {
    int l = level_of(off, L, r);
    for (int t = 0; t < h; ++t) {
      int64_t c;
      if (!draw_col(seed, off, L, r, l, t, &c)) continue;
      int64_t owner = c < r ? c : r;
      int64_t other = c < r ? r : c;
      int64_t pos;
#pragma omp atomic capture
      pos = fill[owner]++;
      ent[pos].j = (int32_t)other;
      ent[pos].v = gauss_half(seed, (uint64_t)r, (uint64_t)t);
      ent[pos].key = (uint64_t)r * 1024u + (uint64_t)t;
    }
  }
  free(fill);

  /* pass 3: sort each owner's segment by (column, key) and keep the first of each column */
  int64_t* ucnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!ucnt) { free(cnt); free(ent); return -2; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    entry_t* s = ent + cnt[i];
    int64_t m = cnt[i + 1] - cnt[i];
    if (m > 1) qsort(s, (size_t)m, sizeof(entry_t), cmp_entry);
    int64_t u = 0;
    for (int64_t a = 0; a < m; ++a) {
      if (u > 0 && s[u - 1].j == s[a].j) continue;
      s[u++] = s[a];
    }
    ucnt[i + 1] = u + 1; /* + diagonal */
  }
  for (int64_t i = 0; i < n; ++i) ucnt[i + 1] += ucnt[i];
  const int64_t nnz = ucnt[n];

  int32_t* col = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
  float* val = (float*)malloc((size_t)nnz * sizeof(float));
  if (!col || !val) { free(cnt); free(ent); free(ucnt); free(col); free(val); return -2; }

  /* pass 4: write the upper CSR, diagonal first in each row */
#pragma omp parallel for schedule(static, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int l = level_of(off, L, i);
    int64_t o = ucnt[i];
    col[o] = (int32_t)i;
    val[o] = (float)(10.0 * l + (2.0 * u01(ctr(seed, S_DIAG, (uint64_t)i, 0)) - 1.0));
    int64_t u = ucnt[i + 1] - ucnt[i] - 1;
    const entry_t* s = ent + cnt[i];
    for (int64_t a = 0; a < u; ++a) {
      col[o + 1 + a] = s[a].j;
      val[o + 1 + a] = s[a].v;
    }
  }
  free(ent);
  free(cnt);

  *n_out = n;
  *nnz_out = nnz;
  *row_ptr_out = ucnt;
  *col_out = col;
  *val_out = val;
  return 0;
}

void levelgen_free(void* p) { free(p); }

int levelgen_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
