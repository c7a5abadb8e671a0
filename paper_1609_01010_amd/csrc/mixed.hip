// Transforms and products of length N = q M, q odd, M a power of two, both
// dividing p - 1: the general-size modular transforms that the library
// generation of section 1 builds on (its references [24, 25, 27] generalise
// the radix).  The odd factors of p - 1 are 3 and 5 for 2013265921, 7 and 17
// for 998244353, 7 for 469762049 and 5 for 167772161.
//
// Since gcd(q, M) = 1 the split needs no twiddles (prime-factor algorithm).
// The index j < N is represented by (j mod q, j mod M) (Chinese remainder
// theorem: Z/N = Z/q x Z/M as rings), and the output index by
// k = (M k1 + q k2) mod N.  Then, with w = w_N,
//   w^{j k} = w_q^{(j mod q) k1} w_M^{(j mod M) k2},
// w_q = w^M and w_M = w^q being the standard roots of orders q and M.  So the
// length-N transform is a length-q transform over j mod q, for each
// j2 = j mod M, followed by q length-M transforms (one per k1), read out at
// the positions (M k1 + q k2) mod N.
//
// For the product, the ring isomorphism alone suffices: the cyclic
// convolution of length N becomes a q x M two-dimensional cyclic
// convolution of the arrays a2[j mod q][j mod M] = a_j.  A length-q transform
// along the first axis (any primitive q-th root) turns it into q independent
// cyclic convolutions of length M (eq. 5, the circular convolution, by the
// convolution theorem), whose results are transformed back along the first
// axis with the factor q^-1.  Acyclic products need N >= la + lb - 1.
//
// Kernels (one thread per j2 < M; all HBM accesses of a wave are contiguous
// except the scatter to (M k1 + q k2) mod N, which has stride q):
//   k_mixed_split: x (flat, zero beyond lx) -> q rows of M: row k1, column
//                  j2 = sum over j = j2 + M t of x_j w_q^{(j mod q) k1}
//   k_mixed_merge: q rows of M -> flat y_j = s * sum_k1 row_k1[j mod M]
//                  w_q^{-(j mod q) k1} for j < ly
//   k_mixed_perm:  q rows of M <-> flat array at (M k1 + q k2) mod N
//
// With r = j2 mod q and m = M mod q, j = j2 + M t has j mod q = (r + m t) mod
// q, so the length-q sum over t has the wave-uniform root w_q^{m k1} and a
// per-lane factor w_q^{r k1}, taken from a table in LDS.  The length-q sums
// pair the terms t and q - t (half the products of the plain sum), and q = 15
// runs as 3 x 5 (prime-factor algorithm).
#include "internal.h"
#include "trace.h"

namespace pm {

constexpr int kMixedMaxQ = 17;

struct MixedRoots {
  uint2 c[kMixedMaxQ];  // (U^e + U^-e) / 2, e < q, U = w_q^{+-m}: the wave-uniform root
  uint2 d[kMixedMaxQ];  // (U^e - U^-e) / 2
  uint2 v[kMixedMaxQ];  // s * w_q^{+-e}, e < q: the per-lane factors (times the scale s)
};

// The length-N transform y_k = sum_t x_t V^{t k} of registers, N odd, with
// V = U^D of order N (U of order Q).  The inputs t and N - t meet V^{tk} and
// V^{-tk}, so with their sum s_t and difference d_t,
//   x_t V^{tk} + x_{N-t} V^{-tk} = s_t (V^{tk} + V^{-tk}) / 2 + d_t (V^{tk} - V^{-tk}) / 2,
// and the output N - k takes the same products with the d terms negated:
// (N - 1)^2 / 2 products in place of (N - 1)^2.  Exponents are reduced at
// compile time; canonical in and out.
template <int Q, int N, int D>
__device__ __forceinline__ void dft_pairs(const Arith<false>& A, const u32 (&x)[N], u32 (&y)[N], const MixedRoots& R) {
  constexpr int H = (N - 1) / 2;
  u32 sm[H + 1], df[H + 1];
  u32 y0 = x[0];
#pragma unroll
  for (int t = 1; t <= H; ++t) {
    sm[t] = A.add(x[t], x[N - t]);
    df[t] = A.subraw(x[t], x[N - t]);  // only multiplied: (0, 2p) is a Shoup input
    y0 = A.add(y0, sm[t]);
  }
  y[0] = y0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    u32 ev = x[0], od = 0;
#pragma unroll
    for (int t = 1; t <= H; ++t) {
      const int e = (D * ((t * k) % N)) % Q;
      ev = A.add(ev, A.mul(sm[t], R.c[e]));
      od = A.add(od, A.mul(df[t], R.d[e]));
    }
    y[k] = A.add(ev, od);
    y[N - k] = A.sub(ev, od);
  }
}

// The length-q transform y_k = sum_t x_t U^{t k} (U of order q).  q = 15 by
// the prime-factor algorithm over 3 x 5 (Good-Thomas): the input t sits at
// (t mod 3, t mod 5), that is t = (10 t1 + 6 t2) mod 15, and the output k at
// k = (5 k1 + 3 k2) mod 15; then t k = 5 t1 k1 + 3 t2 k2 (mod 15), so the
// 15-point transform is five 3-point transforms with root U^5 and three
// 5-point ones with root U^3, no twiddles.
template <int Q>
__device__ __forceinline__ void dft_q(const Arith<false>& A, const u32 (&x)[Q], u32 (&y)[Q], const MixedRoots& R) {
  if constexpr (Q == 15) {
    u32 z[5][3];
#pragma unroll
    for (int t2 = 0; t2 < 5; ++t2) {
      u32 in[3];
#pragma unroll
      for (int t1 = 0; t1 < 3; ++t1) in[t1] = x[(10 * t1 + 6 * t2) % 15];
      dft_pairs<15, 3, 5>(A, in, z[t2], R);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      u32 in[5], out[5];
#pragma unroll
      for (int t2 = 0; t2 < 5; ++t2) in[t2] = z[t2][k1];
      dft_pairs<15, 5, 3>(A, in, out, R);
#pragma unroll
      for (int k2 = 0; k2 < 5; ++k2) y[(5 * k1 + 3 * k2) % 15] = out[k2];
    }
  } else {
    dft_pairs<Q, Q, 1>(A, x, y, R);
  }
}

// blockIdx.y selects the operand: (x0, lx0) into rows0 or (x1, lx1) into rows1
template <int Q>
__global__ void __launch_bounds__(256) k_mixed_split(const u32* __restrict__ x0, long lx0, u32* __restrict__ rows0,
                                                     const u32* __restrict__ x1, long lx1, u32* __restrict__ rows1,
                                                     long M, MixedRoots R, ModP mp, int* err) {
  const u32* __restrict__ x = blockIdx.y ? x1 : x0;
  const long lx = blockIdx.y ? lx1 : lx0;
  u32* __restrict__ rows = blockIdx.y ? rows1 : rows0;
  __shared__ uint2 vt[Q];
  if (threadIdx.x < Q) vt[threadIdx.x] = R.v[threadIdx.x];
  __syncthreads();
  const Arith<false> A(mp);
  for (long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x; j2 < M; j2 += (long)gridDim.x * blockDim.x) {
    u32 v[Q], y[Q];
    bool bad = false;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const long j = j2 + M * t;
      const u32 xv = j < lx ? gld(x + j) : 0u;
      bad |= xv >= mp.p;
      v[t] = xv;
    }
    if (bad) atomicOr(err, 1);
    dft_q<Q>(A, v, y, R);
    // row k1 gets y_k1 * w_q^{r k1}, r = j2 mod q
    const int r = (int)(j2 % Q);
    int e = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      gst(rows + (long)k * M + j2, k == 0 ? y[0] : A.mul(y[k], vt[e]));
      e += r;
      e -= e >= Q ? Q : 0;
    }
  }
}

template <int Q>
__global__ void __launch_bounds__(256) k_mixed_merge(const u32* __restrict__ rows, long M, u32* __restrict__ y,
                                                     long ly, MixedRoots R, ModP mp) {
  __shared__ uint2 vt[Q];
  if (threadIdx.x < Q) vt[threadIdx.x] = R.v[threadIdx.x];
  __syncthreads();
  const Arith<false> A(mp);
  for (long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x; j2 < M; j2 += (long)gridDim.x * blockDim.x) {
    // c_k1 * s * w_q^{-r k1}, then the length-q sum over k1 with root w_q^{-m}
    const int r = (int)(j2 % Q);
    u32 c[Q], out[Q];
    int e = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      c[k] = A.mul(gld(rows + (long)k * M + j2), vt[e]);
      e += r;
      e -= e >= Q ? Q : 0;
    }
    dft_q<Q>(A, c, out, R);
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const long j = j2 + M * t;
      if (j < ly) gst(y + j, out[t]);
    }
  }
}

// to_flat: flat[(M k1 + q k2) mod N] = rows[k1][k2]; else the reverse
template <int Q>
__global__ void __launch_bounds__(256) k_mixed_perm(const u32* __restrict__ in, long M, u32* __restrict__ out,
                                                    int to_flat) {
  const long N = M * Q;
  for (long k2 = (long)blockIdx.x * blockDim.x + threadIdx.x; k2 < M; k2 += (long)gridDim.x * blockDim.x) {
    long pos = (long)Q * k2;  // < N
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {
      if (to_flat)
        gst(out + pos, gld(in + (long)k1 * M + k2));
      else
        gst(out + (long)k1 * M + k2, gld(in + pos));
      pos += M;
      pos -= pos >= N ? N : 0;
    }
  }
}

// Descriptors of the q row products, so that each pass of the circular
// products runs once over all rows (blockIdx.z selects the row): job r is
// `base` with its operands and result advanced by r * stride words and its
// four-step workspace by r * tstride words.
__global__ void k_row_jobs(ConvJob base, long stride, long tstride, int q, ConvJob* __restrict__ out) {
  const int r = threadIdx.x;
  if (r >= q) return;
  ConvJob J = base;
  J.a = (const u32*)base.a + r * stride;
  J.b = (const u32*)base.b + r * stride;
  J.c = base.c + r * stride;
  if (base.Ta) J.Ta = base.Ta + r * tstride;
  if (base.Tb) J.Tb = base.Tb + r * tstride;
  out[r] = J;
}

hipError_t launch_row_jobs(const ConvJob& base, long stride, long tstride, int q, ConvJob* out, hipStream_t s) {
  return launch("row_jobs", k_row_jobs, 1, 64, 0, s, base, stride, tstride, q, out);
}

static unsigned mixed_blocks(long M) {
  long b = (M + 255) / 256;
  return (unsigned)(b > 4096 ? 4096 : b);
}

// roots for direction dir (0: w_q, 1: w_q^-1) and per-lane scale s
static MixedRoots mixed_roots(const PrimeInfo& P, int q, long M, int dir, u32 scale) {
  MixedRoots R{};
  u32 w = h_powmod(P.g, (P.p - 1) / (u32)q, P.p);
  if (dir) w = h_inv(w, P.p);
  const u32 wm = h_powmod(w, (u64)(M % q), P.p);
  const u32 half = (P.p + 1) / 2;  // 2^-1 mod p
  u32 up[kMixedMaxQ];
  u32 a = 1, b = scale % P.p;
  for (int e = 0; e < q; ++e) {
    up[e] = a;
    R.v[e] = h_shoup(b, P.p);
    a = h_mulmod(a, wm, P.p);
    b = h_mulmod(b, w, P.p);
  }
  for (int e = 0; e < q; ++e) {
    const u32 x = up[e], y = up[(q - e) % q];  // U^e, U^-e
    R.c[e] = h_shoup(h_mulmod((x + y) % P.p, half, P.p), P.p);
    R.d[e] = h_shoup(h_mulmod((x + P.p - y) % P.p, half, P.p), P.p);
  }
  return R;
}

bool mixed_q_supported(int q) { return q == 3 || q == 5 || q == 7 || q == 15 || q == 17; }

#define PM_MIXED_DISPATCH(q, CALL) \
  switch (q) {                     \
    case 3: CALL(3);               \
    case 5: CALL(5);               \
    case 7: CALL(7);               \
    case 15: CALL(15);             \
    case 17: CALL(17);             \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_mixed_split(const u32* x0, long lx0, u32* rows0, const u32* x1, long lx1, u32* rows1, int q, long M,
                              int pidx, int* err, hipStream_t s) {
  const PrimeInfo& P = prime_info(pidx);
  const MixedRoots R = mixed_roots(P, q, M, 0, 1);
  const ModP mp = modp_of(P);
  const dim3 grid(mixed_blocks(M), x1 ? 2 : 1);
#define PM_SPLIT(Q) \
  return launch("mixed_split", k_mixed_split<Q>, grid, 256, 0, s, x0, lx0, rows0, x1, lx1, rows1, M, R, mp, err)
  PM_MIXED_DISPATCH(q, PM_SPLIT)
#undef PM_SPLIT
}

hipError_t launch_mixed_merge(const u32* rows, int q, long M, u32* y, long ly, int pidx, hipStream_t s) {
  const PrimeInfo& P = prime_info(pidx);
  const MixedRoots R = mixed_roots(P, q, M, 1, h_inv((u32)q, P.p));
  const ModP mp = modp_of(P);
#define PM_MERGE(Q) return launch("mixed_merge", k_mixed_merge<Q>, mixed_blocks(M), 256, 0, s, rows, M, y, ly, R, mp)
  PM_MIXED_DISPATCH(q, PM_MERGE)
#undef PM_MERGE
}

hipError_t launch_mixed_perm(const u32* in, int q, long M, u32* out, int to_flat, hipStream_t s) {
#define PM_PERM(Q) return launch("mixed_perm", k_mixed_perm<Q>, mixed_blocks(M), 256, 0, s, in, M, out, to_flat)
  PM_MIXED_DISPATCH(q, PM_PERM)
#undef PM_PERM
}

#undef PM_MIXED_DISPATCH

}  // namespace pm
