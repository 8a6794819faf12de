/*
 * Exact k-nearest-neighbour lists of integer points under the squared
 * Euclidean distance, ties broken towards the smaller point index.
 *
 * Input generator only (the single-cell-shaped kNN workload): nothing here
 * is part of the consensus method.  The points are small integers, so every
 * dot product, squared norm and distance is an integer below 2^24 and is
 * computed exactly in single precision whatever the order of the sums; the
 * result is therefore the same as any other exact evaluation (the torch
 * path in graph.py, on a CPU or a GPU).
 *
 * Points are visited in increasing index for every query, so a candidate
 * whose distance equals the current k-th best never displaces it (its index
 * is larger): the strict comparison below is the (distance, index) order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <immintrin.h>

#define QB 8          /* queries per register block */
#define TILE 4096     /* points per cache tile */
#define SUPER 256     /* queries per task */

typedef struct {
  int64_t key[64]; /* (distance << 32) | index, ascending */
  int32_t count;
} toplist;

static void insert(toplist* t, int kk, int64_t key) {
  int c = t->count;
  if (c == kk) {
    if (key >= t->key[kk - 1]) return;
    c = kk - 1;
  }
  int j = c;
  while (j > 0 && t->key[j - 1] > key) {
    t->key[j] = t->key[j - 1];
    --j;
  }
  t->key[j] = key;
  if (t->count < kk) t->count += 1;
}

static float threshold(const toplist* t, int kk) {
  return t->count < kk ? INFINITY : (float)(t->key[kk - 1] >> 32);
}


#define TILE_ARGS                                                                              \
  const float *X, const float *SQ, const float *Q, const float *QS, int64_t npad, int dim,   \
      int kk, int64_t q0, int qb, int nb, int64_t p0, int64_t p1, toplist *tl, float *thr

/* One tile of points against one block of QB queries. */
__attribute__((target("avx512f,fma"))) static void tile_avx512(TILE_ARGS) {
  for (int64_t p = p0; p < p1; p += 16) {
    __m512 acc[QB];
    for (int r = 0; r < QB; ++r) acc[r] = _mm512_setzero_ps();
    for (int d = 0; d < dim; ++d) {
      const __m512 xv = _mm512_loadu_ps(X + (int64_t)d * npad + p);
      for (int r = 0; r < QB; ++r)
        acc[r] = _mm512_fmadd_ps(_mm512_set1_ps(Q[(qb + r) * dim + d]), xv, acc[r]);
    }
    const __m512 sp = _mm512_loadu_ps(SQ + p);
    for (int r = 0; r < nb; ++r) {
      const __m512 dist = _mm512_fmadd_ps(_mm512_set1_ps(-2.f), acc[r],
                                          _mm512_add_ps(sp, _mm512_set1_ps(QS[qb + r])));
      __mmask16 m = _mm512_cmp_ps_mask(dist, _mm512_set1_ps(thr[r]), _CMP_LT_OQ);
      if (!m) continue;
      float dv[16];
      _mm512_storeu_ps(dv, dist);
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1;
        const int64_t j = p + b;
        if (j >= p1 || j == q0 + qb + r) continue;
        insert(&tl[qb + r], kk, ((int64_t)dv[b] << 32) | j);
      }
      thr[r] = threshold(&tl[qb + r], kk);
    }
  }
}

static void tile_scalar(TILE_ARGS) {
  for (int64_t p = p0; p < p1; ++p) {
    for (int r = 0; r < nb; ++r) {
      float acc = 0.f;
      for (int d = 0; d < dim; ++d) acc += Q[(qb + r) * dim + d] * X[(int64_t)d * npad + p];
      const float dist = (SQ[p] + QS[qb + r]) - 2.f * acc;
      if (dist < thr[r] && p != q0 + qb + r) {
        insert(&tl[qb + r], kk, ((int64_t)dist << 32) | p);
        thr[r] = threshold(&tl[qb + r], kk);
      }
    }
  }
}

/* Returns 0, or -1 for arguments outside the exact range, -2 on allocation
 * failure.  out[q * kk + r] is the r-th nearest point of q (q excluded),
 * -1 where fewer than kk other points exist. */
int knn_exact(const int32_t* pts, int64_t n, int32_t dim, int32_t kk, int32_t* out) {
  if (n < 0 || dim < 1 || dim > 64 || kk < 1 || kk > 64 || n >= ((int64_t)1 << 31)) return -1;
  int64_t maxabs = 0;
  for (int64_t j = 0; j < n * dim; ++j) {
    int64_t a = pts[j] < 0 ? -(int64_t)pts[j] : pts[j];
    if (a > maxabs) maxabs = a;
  }
  /* every distance, norm and partial dot product below 2^24 */
  if (4 * (int64_t)dim * maxabs * maxabs >= ((int64_t)1 << 24)) return -1;
  const int64_t npad = (n + 15) / 16 * 16 + 16;
  float* X = (float*)malloc(sizeof(float) * (size_t)npad * (size_t)dim);
  float* SQ = (float*)malloc(sizeof(float) * (size_t)npad);
  if (!X || !SQ) {
    free(X);
    free(SQ);
    return -2;
  }
  for (int64_t j = 0; j < npad; ++j) {
    int64_t s = 0;
    for (int d = 0; d < dim; ++d) {
      const int64_t x = j < n ? pts[j * dim + d] : 0;
      X[(int64_t)d * npad + j] = (float)x;
      s += x * x;
    }
    SQ[j] = j < n ? (float)s : INFINITY;
  }
  const int use_avx512 = __builtin_cpu_supports("avx512f");
  const int64_t nsuper = (n + SUPER - 1) / SUPER;
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t sb = 0; sb < nsuper; ++sb) {
    const int64_t q0 = sb * SUPER;
    const int nq = (int)(n - q0 < SUPER ? n - q0 : SUPER);
    toplist* tl = (toplist*)calloc((size_t)SUPER, sizeof(toplist));
    float* Q = (float*)calloc((size_t)SUPER * (size_t)dim, sizeof(float));
    float* QS = (float*)calloc((size_t)SUPER, sizeof(float));
    if (!tl || !Q || !QS) {
      free(tl);
      free(Q);
      free(QS);
#pragma omp atomic write
      failed = 1;
      continue;
    }
    for (int q = 0; q < nq; ++q) {
      for (int d = 0; d < dim; ++d) Q[q * dim + d] = X[(int64_t)d * npad + q0 + q];
      QS[q] = SQ[q0 + q];
    }
    for (int64_t p0 = 0; p0 < n; p0 += TILE) {
      const int64_t p1 = p0 + TILE < n ? p0 + TILE : n;
      for (int qb = 0; qb < nq; qb += QB) {
        const int nb = nq - qb < QB ? nq - qb : QB;
        float thr[QB];
        for (int r = 0; r < QB; ++r) thr[r] = r < nb ? threshold(&tl[qb + r], kk) : -INFINITY;
        if (use_avx512)
          tile_avx512(X, SQ, Q, QS, npad, dim, kk, q0, qb, nb, p0, p1, tl, thr);
        else
          tile_scalar(X, SQ, Q, QS, npad, dim, kk, q0, qb, nb, p0, p1, tl, thr);
      }
    }
    for (int q = 0; q < nq; ++q)
      for (int r = 0; r < kk; ++r)
        out[(q0 + q) * kk + r] = r < tl[q].count ? (int32_t)(tl[q].key[r] & 0xffffffff) : -1;
    free(tl);
    free(Q);
    free(QS);
  }
  free(X);
  free(SQ);
  return failed ? -2 : 0;
}
