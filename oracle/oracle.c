/*
 * Reference computations for the modular polynomial product, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this file;
 * only the tests, the smoke check and the benchmark's CPU baseline do.  It
 * shares no code with the GPU path.
 *
 * Every routine is the textbook definition, written for clarity:
 *   - orc_polymul:        c_k = sum_{i+j=k} a_i b_j mod p      (Def. 2, eq. 2;
 *                         the same sum as the linear convolution, Def. 3, eq. 3)
 *   - orc_polymul_sample: the same sum, for a chosen set of output indices k
 *   - orc_cyclic:         (u (*) v)_i = sum_k u_k v_{(i-k) mod N} (Def. 4, eq. 5)
 *   - orc_negacyclic:     the product in R[x]/(x^N + 1), the second factor of
 *                         eq. 13: sum_{k<=i} u_k v_{i-k} - sum_{k>i} u_k v_{N+i-k}
 *   - orc_ntt:            X_k = sum_j x_j w^{jk} (evaluation at w^0..w^{N-1},
 *                         section 3, convolution theorem), by the iterative
 *                         radix-2 Cooley-Tukey algorithm; inverse scaled by N^-1
 *   - orc_eval:           a(x) mod p by Horner's rule
 * Arithmetic is exact: 64-bit products, 128-bit accumulation.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a * b) % p); }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  b %= p;
  while (e) {
    if (e & 1) r = mulmod(r, b, p);
    b = mulmod(b, b, p);
    e >>= 1;
  }
  return r;
}

/* c[k] = sum_{i+j=k} a[i] b[j] mod p, k = 0 .. la+lb-2 */
void orc_polymul(const uint32_t* a, int64_t la, const uint32_t* b, int64_t lb, uint32_t p, uint32_t* c) {
  int64_t lc = la + lb - 1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < lc; ++k) {
    int64_t i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0;
    int64_t i1 = k < la - 1 ? k : la - 1;
    u128 acc = 0;
    for (int64_t i = i0; i <= i1; ++i) acc += (uint64_t)a[i] * b[k - i];
    c[k] = (uint32_t)(acc % p);
  }
}

/* the same sum for the output indices ks[0..nk) only */
void orc_polymul_sample(const uint32_t* a, int64_t la, const uint32_t* b, int64_t lb, uint32_t p,
                        const int64_t* ks, int64_t nk, uint32_t* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nk; ++t) {
    int64_t k = ks[t];
    int64_t i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0;
    int64_t i1 = k < la - 1 ? k : la - 1;
    u128 acc = 0;
    for (int64_t i = i0; i <= i1; ++i) acc += (uint64_t)a[i] * b[k - i];
    out[t] = (uint32_t)(acc % p);
  }
}

/* circular convolution of two length-N vectors mod p */
void orc_cyclic(const uint32_t* u, const uint32_t* v, int64_t n, uint32_t p, uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    u128 acc = 0;
    for (int64_t k = 0; k < n; ++k) acc += (uint64_t)u[k] * v[((i - k) % n + n) % n];
    out[i] = (uint32_t)(acc % p);
  }
}

void orc_negacyclic(const uint32_t* u, const uint32_t* v, int64_t n, uint32_t p, uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    u128 pos = 0, neg = 0;
    for (int64_t k = 0; k <= i; ++k) pos += (uint64_t)u[k] * v[i - k];
    for (int64_t k = i + 1; k < n; ++k) neg += (uint64_t)u[k] * v[n + i - k];
    out[i] = (uint32_t)(((pos % p) + p - (neg % p)) % p);
  }
}

/* Horner evaluation of a(x) mod p */
uint32_t orc_eval(const uint32_t* a, int64_t la, uint32_t p, uint32_t x) {
  uint64_t r = 0;
  for (int64_t i = la - 1; i >= 0; --i) r = (mulmod(r, x, p) + a[i]) % p;
  return (uint32_t)r;
}

/* In-place transform of length n (a power of two) with root w = g^((p-1)/n),
 * or w^-1 and a final factor n^-1 when inverse != 0.  Natural order in and out. */
int orc_ntt(uint32_t* x, int64_t n, uint32_t p, uint32_t g, int inverse) {
  if (n < 1 || (n & (n - 1))) return -1;
  if ((p - 1) % (uint64_t)n) return -2;
  /* bit-reversal permutation */
  for (int64_t i = 1, j = 0; i < n; ++i) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j |= bit;
    if (i < j) {
      uint32_t t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
  /* butterflies: len = 2, 4, ..., n */
  for (int64_t len = 2; len <= n; len <<= 1) {
    uint64_t w = powmod(g, (p - 1) / (uint64_t)len, p);
    if (inverse) w = powmod(w, p - 2, p);
    int64_t half = len >> 1;
    /* powers of w for this level */
    uint64_t* wp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)half);
    if (!wp) return -3;
    wp[0] = 1;
    for (int64_t t = 1; t < half; ++t) wp[t] = mulmod(wp[t - 1], w, p);
#pragma omp parallel for schedule(static) if (n >= (1 << 16))
    for (int64_t s = 0; s < n; s += len) {
      for (int64_t t = 0; t < half; ++t) {
        uint64_t u = x[s + t];
        uint64_t v = mulmod(x[s + t + half], wp[t], p);
        x[s + t] = (uint32_t)((u + v) % p);
        x[s + t + half] = (uint32_t)((u + p - v) % p);
      }
    }
    free(wp);
  }
  if (inverse) {
    uint64_t ninv = powmod((uint64_t)n % p, p - 2, p);
    for (int64_t i = 0; i < n; ++i) x[i] = (uint32_t)mulmod(x[i], ninv, p);
  }
  return 0;
}

/* c = a * b mod p via zero padding to the next power of two >= la+lb-1 and
 * orc_ntt (eq. 12); the scratch arrays are allocated here. */
int orc_polymul_ntt(const uint32_t* a, int64_t la, const uint32_t* b, int64_t lb, uint32_t p, uint32_t g,
                    uint32_t* c) {
  int64_t lc = la + lb - 1, n = 1;
  while (n < lc) n <<= 1;
  uint32_t* fa = (uint32_t*)calloc((size_t)n, 4);
  uint32_t* fb = (uint32_t*)calloc((size_t)n, 4);
  if (!fa || !fb) {
    free(fa);
    free(fb);
    return -3;
  }
  memcpy(fa, a, (size_t)la * 4);
  memcpy(fb, b, (size_t)lb * 4);
  int rc = orc_ntt(fa, n, p, g, 0);
  if (!rc) rc = orc_ntt(fb, n, p, g, 0);
  if (!rc) {
    for (int64_t i = 0; i < n; ++i) fa[i] = (uint32_t)mulmod(fa[i], fb[i], p);
    rc = orc_ntt(fa, n, p, g, 1);
  }
  if (!rc) memcpy(c, fa, (size_t)lc * 4);
  free(fa);
  free(fb);
  return rc;
}
