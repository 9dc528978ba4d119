/*
 * Plain C Bareiss determinant over arbitrary-precision integers.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle, never linked into or
 * called by the GPU library.  It exists because the Python-int version of
 * the same definition takes hours at n = 1024.
 *
 * Definition written out (the exact integer det(A) that the paper's
 * Chinese-remaindering loop reconstructs, Section 2.1): fraction-free
 * Gaussian elimination.  prev = 1; for k = 0..n-2: if a_kk = 0 swap in the
 * first lower row with a non-zero entry in column k (flip the sign), or
 * return 0 if there is none; then for i, j > k:
 *     a_ij <- (a_kk a_ij - a_ik a_kj) / prev      (exact division)
 * and prev <- a_kk.  det = sign * a_{n-1,n-1}.
 *
 * Big integers: sign + magnitude in base 2^32 limbs, schoolbook multiply,
 * Knuth's long division (algorithm D) with a remainder check.  The rows
 * i > k of one elimination step are independent and split over OpenMP
 * threads; that changes no arithmetic.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int sign;      /* -1, 0, +1 */
  int len;       /* limbs in use; 0 for zero */
  int cap;
  uint32_t *d;   /* little-endian magnitude */
} big;

static int big_reserve(big *x, int n) {
  if (x->cap >= n) return 0;
  int c = x->cap ? x->cap : 4;
  while (c < n) c *= 2;
  uint32_t *p = (uint32_t *)realloc(x->d, (size_t)c * sizeof(uint32_t));
  if (!p) return -1;
  x->d = p;
  x->cap = c;
  return 0;
}

static void big_trim(big *x) {
  while (x->len > 0 && x->d[x->len - 1] == 0) x->len--;
  if (x->len == 0) x->sign = 0;
}

static int big_set_i64(big *x, int64_t v) {
  if (big_reserve(x, 2)) return -1;
  uint64_t m = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
  x->sign = v < 0 ? -1 : (v > 0 ? 1 : 0);
  x->d[0] = (uint32_t)m;
  x->d[1] = (uint32_t)(m >> 32);
  x->len = 2;
  big_trim(x);
  return 0;
}

static int big_copy(big *dst, const big *src) {
  if (big_reserve(dst, src->len > 0 ? src->len : 1)) return -1;
  memcpy(dst->d, src->d, (size_t)src->len * sizeof(uint32_t));
  dst->len = src->len;
  dst->sign = src->sign;
  return 0;
}

/* out = a * b (out must not alias a or b) */
static int big_mul(big *out, const big *a, const big *b) {
  if (a->sign == 0 || b->sign == 0) { out->sign = 0; out->len = 0; return 0; }
  int n = a->len + b->len;
  if (big_reserve(out, n)) return -1;
  memset(out->d, 0, (size_t)n * sizeof(uint32_t));
  for (int i = 0; i < a->len; i++) {
    uint64_t carry = 0, ai = a->d[i];
    for (int j = 0; j < b->len; j++) {
      uint64_t t = ai * b->d[j] + out->d[i + j] + carry;
      out->d[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    out->d[i + b->len] = (uint32_t)carry;
  }
  out->len = n;
  out->sign = a->sign * b->sign;
  big_trim(out);
  return 0;
}

/* compare magnitudes */
static int mag_cmp(const big *a, const big *b) {
  if (a->len != b->len) return a->len < b->len ? -1 : 1;
  for (int i = a->len - 1; i >= 0; i--)
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  return 0;
}

/* out = |a| + |b| */
static int mag_add(big *out, const big *a, const big *b) {
  const big *x = a->len >= b->len ? a : b, *y = a->len >= b->len ? b : a;
  if (big_reserve(out, x->len + 1)) return -1;
  uint64_t carry = 0;
  for (int i = 0; i < x->len; i++) {
    uint64_t t = (uint64_t)x->d[i] + (i < y->len ? y->d[i] : 0) + carry;
    out->d[i] = (uint32_t)t;
    carry = t >> 32;
  }
  out->d[x->len] = (uint32_t)carry;
  out->len = x->len + 1;
  return 0;
}

/* out = |a| - |b|, requires |a| >= |b| */
static int mag_sub(big *out, const big *a, const big *b) {
  if (big_reserve(out, a->len > 0 ? a->len : 1)) return -1;
  int64_t borrow = 0;
  for (int i = 0; i < a->len; i++) {
    int64_t t = (int64_t)a->d[i] - (i < b->len ? (int64_t)b->d[i] : 0) - borrow;
    borrow = t < 0;
    out->d[i] = (uint32_t)(t + (borrow ? ((int64_t)1 << 32) : 0));
  }
  out->len = a->len;
  return 0;
}

/* out = a - b (out must not alias a or b) */
static int big_sub(big *out, const big *a, const big *b) {
  if (b->sign == 0) return big_copy(out, a);
  if (a->sign == 0) { if (big_copy(out, b)) return -1; out->sign = -out->sign; return 0; }
  if (a->sign != b->sign) {           /* a - b = sign(a) (|a| + |b|) */
    if (mag_add(out, a, b)) return -1;
    out->sign = a->sign;
  } else {
    int c = mag_cmp(a, b);
    if (c == 0) { out->sign = 0; out->len = 0; return 0; }
    if (c > 0) { if (mag_sub(out, a, b)) return -1; out->sign = a->sign; }
    else { if (mag_sub(out, b, a)) return -1; out->sign = -a->sign; }
  }
  big_trim(out);
  return 0;
}

static int clz32(uint32_t x) { return x ? __builtin_clz(x) : 32; }

/*
 * q = a / b exactly.  Knuth's algorithm D on magnitudes (normalise so the
 * divisor's top limb has its high bit set, estimate each quotient limb from
 * the top two remainder limbs, correct by at most two, multiply-subtract,
 * add back on a negative result).  Returns 1 if the remainder is non-zero.
 * un, vn: caller scratch bigs.
 */
static int big_divexact(big *q, const big *a, const big *b, big *un, big *vn) {
  if (b->sign == 0) return -1;
  if (a->sign == 0) { q->sign = 0; q->len = 0; return 0; }
  int m = a->len, n = b->len;
  if (m < n) return 1;                          /* |a| < |b|, a != 0 */
  if (big_reserve(q, m - n + 1)) return -1;
  if (n == 1) {
    uint64_t r = 0, v = b->d[0];
    for (int i = m - 1; i >= 0; i--) {
      uint64_t cur = (r << 32) | a->d[i];
      q->d[i] = (uint32_t)(cur / v);
      r = cur % v;
    }
    q->len = m;
    q->sign = a->sign * b->sign;
    big_trim(q);
    return r != 0;
  }
  int s = clz32(b->d[n - 1]);
  if (big_reserve(vn, n) || big_reserve(un, m + 1)) return -1;
  for (int i = n - 1; i > 0; i--)
    vn->d[i] = s ? (b->d[i] << s) | (b->d[i - 1] >> (32 - s)) : b->d[i];
  vn->d[0] = b->d[0] << s;
  un->d[m] = s ? a->d[m - 1] >> (32 - s) : 0;
  for (int i = m - 1; i > 0; i--)
    un->d[i] = s ? (a->d[i] << s) | (a->d[i - 1] >> (32 - s)) : a->d[i];
  un->d[0] = a->d[0] << s;
  const uint64_t B = (uint64_t)1 << 32;
  for (int j = m - n; j >= 0; j--) {
    uint64_t num = ((uint64_t)un->d[j + n] << 32) | un->d[j + n - 1];
    uint64_t qhat = num / vn->d[n - 1];
    uint64_t rhat = num % vn->d[n - 1];
    while (qhat >= B || qhat * vn->d[n - 2] > ((rhat << 32) | un->d[j + n - 2])) {
      qhat--;
      rhat += vn->d[n - 1];
      if (rhat >= B) break;
    }
    int64_t borrow = 0;
    uint64_t carry = 0;
    for (int i = 0; i < n; i++) {
      uint64_t p = qhat * vn->d[i] + carry;
      carry = p >> 32;
      int64_t t = (int64_t)un->d[i + j] - (int64_t)(p & 0xffffffffu) - borrow;
      borrow = t < 0;
      un->d[i + j] = (uint32_t)t;
    }
    int64_t t = (int64_t)un->d[j + n] - (int64_t)carry - borrow;
    un->d[j + n] = (uint32_t)t;
    if (t < 0) {                                  /* add back */
      qhat--;
      uint64_t c = 0;
      for (int i = 0; i < n; i++) {
        uint64_t u = (uint64_t)un->d[i + j] + vn->d[i] + c;
        un->d[i + j] = (uint32_t)u;
        c = u >> 32;
      }
      un->d[j + n] = (uint32_t)((uint64_t)un->d[j + n] + c);
    }
    q->d[j] = (uint32_t)qhat;
  }
  q->len = m - n + 1;
  q->sign = a->sign * b->sign;
  big_trim(q);
  for (int i = 0; i < n; i++)
    if (un->d[i]) return 1;                      /* remainder must be zero */
  return 0;
}

static void big_free(big *x) { free(x->d); x->d = NULL; x->cap = x->len = 0; }

/*
 * det(A) for a row-major n x n int64 matrix.  On success (return 0) the
 * magnitude is written to mag[0..*out_len) (little-endian base 2^32) and
 * the sign (-1, 0, +1) to *out_sign.  Returns 1 if cap is too small (then
 * *out_len holds the size needed), -1 on allocation failure, -2 if a
 * division was not exact (cannot happen for a correct elimination).
 */
int oracle_bareiss_det(const int64_t *A, int n, int nthreads, uint32_t *mag, int cap,
                       int *out_len, int *out_sign) {
  *out_len = 0;
  *out_sign = 1;
  if (n == 0) {
    if (cap < 1) { *out_len = 1; return 1; }
    mag[0] = 1;
    *out_len = 1;
    return 0;
  }
  big **M = (big **)malloc((size_t)n * sizeof(big *));
  if (!M) return -1;
  int status = 0;
  for (int i = 0; i < n; i++) {
    M[i] = (big *)calloc((size_t)n, sizeof(big));
    if (!M[i]) return -1;
    for (int j = 0; j < n; j++)
      if (big_set_i64(&M[i][j], A[(size_t)i * n + j])) return -1;
  }
  int sign = 1;
  big prev = {0, 0, 0, NULL};
  big_set_i64(&prev, 1);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  for (int k = 0; k < n - 1 && status == 0; k++) {
    if (M[k][k].sign == 0) {
      int i;
      for (i = k + 1; i < n; i++)
        if (M[i][k].sign != 0) break;
      if (i == n) { sign = 0; break; }
      big *t = M[k]; M[k] = M[i]; M[i] = t;
      sign = -sign;
    }
    const big *akk = &M[k][k];
#pragma omp parallel
    {
      big t1 = {0, 0, 0, NULL}, t2 = {0, 0, 0, NULL}, t3 = {0, 0, 0, NULL};
      big un = {0, 0, 0, NULL}, vn = {0, 0, 0, NULL};
#pragma omp for schedule(dynamic, 1)
      for (int i = k + 1; i < n; i++) {
        big *rowi = M[i];
        const big *aik = &rowi[k];
        for (int j = k + 1; j < n; j++) {
          int e = big_mul(&t1, akk, &rowi[j]);
          e |= big_mul(&t2, aik, &M[k][j]);
          e |= big_sub(&t3, &t1, &t2);
          int r = e ? -1 : big_divexact(&rowi[j], &t3, &prev, &un, &vn);
          if (r) {
#pragma omp atomic write
            status = r < 0 ? -1 : -2;
          }
        }
      }
      big_free(&t1); big_free(&t2); big_free(&t3); big_free(&un); big_free(&vn);
    }
    for (int i = k + 1; i < n; i++) big_free(&M[i][k]);
    if (big_copy(&prev, akk)) status = -1;
  }
  if (status == 0) {
    const big *r = &M[n - 1][n - 1];
    if (sign == 0 || r->sign == 0) {
      *out_sign = 0;
      *out_len = 0;
    } else if (r->len > cap) {
      *out_len = r->len;
      status = 1;
    } else {
      memcpy(mag, r->d, (size_t)r->len * sizeof(uint32_t));
      *out_len = r->len;
      *out_sign = sign * r->sign;
    }
  }
  for (int i = 0; i < n; i++) {
    for (int j = 0; j < n; j++) big_free(&M[i][j]);
    free(M[i]);
  }
  free(M);
  big_free(&prev);
  return status;
}
