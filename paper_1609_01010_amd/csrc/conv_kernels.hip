// Convolution kernels: the defining sum for tiny products, the one-work-group
// LDS-resident convolution, and the three passes of the four-step convolution.
//
// The product is computed by the convolution theorem (Theorem 1, eq. 10):
// forward transforms of both zero-padded operands (eq. 12; the padding is
// never read from memory), the pointwise product (the operator P of eq. 11),
// the inverse transform, and the scaling by the inverse length.  With
// truncation (eq. 14) only the first n' >= len_a + len_b - 1 bit-reversed
// transform values are formed, multiplied and inverted.
//
// Four-step split used throughout, for L = R * C:
//   input index  j = C j1 + j2   (j1 < R: column position, j2 < C: column)
//   output index k = k1 + R k2
//   X_{k1 + R k2} = sum_{j2} w_C^{j2 k2} w_L^{j2 k1} sum_{j1} x_{C j1 + j2} w_R^{j1 k1}
// Column pass: length-R transforms of the columns (bit-reversed out).  Row
// pass: row t holds k1 = rev(t); twiddle by w_L^{j2 k1}, length-C transform,
// and for the convolution the pointwise product and the inverse, untwiddled.
// Truncating to rows t < m keeps the first m C bit-reversed outputs: the TFT
// with granularity C (relaxed, as the paper's library relaxes its breakdown).
#include "internal.h"

namespace pm {

// ---------------------------------------------------------------------------
// the defining sum c_k = sum_{i+j=k} a_i b_j (Def. 2) for products with < 64
// outputs: one thread per output coefficient

template <bool LAZY>
__global__ void __launch_bounds__(64) k_direct(const u32* __restrict__ a, int la, const u32* __restrict__ b, int lb,
                                              u32* __restrict__ c, ModP mp, int* err) {
  const int k = threadIdx.x;
  const int lc = la + lb - 1;
  if (k >= lc) return;
  u64 acc = 0;  // < 64 terms each below 2^31
  const int i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0;
  const int i1 = k < la - 1 ? k : la - 1;
  for (int i = i0; i <= i1; ++i) {
    const u32 x = a[i], y = b[k - i];
    if (x >= mp.p || y >= mp.p) atomicOr(err, 1);
    acc += (u64)x * y % mp.p;
  }
  c[k] = (u32)(acc % mp.p);
}

hipError_t launch_direct(const u32* a, long la, const u32* b, long lb, u32* c, int pidx, int* err, hipStream_t s) {
  const PrimeInfo& P = prime_info(pidx);
  const ModP mp = modp_of(P);
  if (P.lazy)
    k_direct<true><<<1, 64, 0, s>>>(a, (int)la, b, (int)lb, c, mp, err);
  else
    k_direct<false><<<1, 64, 0, s>>>(a, (int)la, b, (int)lb, c, mp, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// one work-group per product, everything in LDS (L = 2^LN <= 2^14).
// The first round (radix RA over the top log2 RA index bits) is done in
// registers straight from global memory and keeps the first ma of its RA
// output blocks; the remaining rounds transform those blocks in LDS.

template <int LN, int LRA, int LQ, bool LAZY>
__global__ void __launch_bounds__(1024) k_lds_conv(const u32* __restrict__ a, int la, const u32* __restrict__ b, int lb,
                                                   u32* __restrict__ c, int lc, int ma, ModP mp, PrimeTables T,
                                                   uint2 sc, int* err) {
  constexpr int N = 1 << LN;
  constexpr int RA = 1 << LRA;
  constexpr int LS = LN - LRA;
  constexpr int S = 1 << LS;
  extern __shared__ u32 sm[];
  u32* sa = sm;
  u32* sb = sm + N;
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x, nthr = blockDim.x;
  bool bad = false;

  for (int j = tid; j < S; j += nthr) {
    uint2 tw[RA];
    if constexpr (S > 1) {
#pragma unroll
      for (int t = 1; t < RA; ++t) tw[t] = T.pf[N + j * (int)(__brev((u32)t) >> (32 - LRA))];
    }
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const u32* in = op ? b : a;
      const int len = op ? lb : la;
      u32* out = op ? sb : sa;
      u32 x[RA];
#pragma unroll
      for (int s = 0; s < RA; ++s) {
        const int pos = j + S * s;
        x[s] = pos < len ? in[pos] : 0u;
        bad |= x[s] >= mp.p;
      }
      dif_reg<RA>(A, x, T.pf);
#pragma unroll
      for (int t = 0; t < RA; ++t) {
        if (t < ma) {
          u32 v = x[t];
          if constexpr (S > 1) {
            if (t > 0) v = A.mul(v, tw[t]);
          }
          out[j + S * t] = v;
        }
      }
    }
  }
  if (bad) atomicOr(err, 1);
  __syncthreads();
  const int nel = ma * S;
  u32* bufs[2] = {sa, sb};
  dif_lds<LS, LQ, LAZY, 2>(A, bufs, nel, T.pf, tid, nthr);
  for (int i = tid; i < nel; i += nthr) sa[i] = A.mul(A.mont(sa[i], sb[i]), sc);
  __syncthreads();
  dit_lds<LS, LQ, LAZY>(A, sa, nel, T.pi, tid, nthr);
  for (int j = tid; j < S; j += nthr) {
    u32 x[RA];
#pragma unroll
    for (int t = 0; t < RA; ++t) {
      u32 v = 0;
      if (t < ma) {
        v = sa[j + S * t];
        if constexpr (S > 1) {
          if (t > 0) v = A.mul(v, T.pi[N + j * (int)(__brev((u32)t) >> (32 - LRA))]);
        }
      }
      x[t] = v;
    }
    inv_column<RA, LAZY>(A, x, ma, T);
#pragma unroll
    for (int s = 0; s < RA; ++s) {
      const int pos = j + S * s;
      if (s < ma && pos < lc) c[pos] = A.canon(x[s]);
    }
  }
}

template <int LN, int LRA, bool LAZY>
static hipError_t lds_conv_inst(const Plan& P, const u32* a, long la, const u32* b, long lb, u32* c, long lc,
                                const ModP& mp, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  constexpr int N = 1 << LN;
  int nthr = N / 16;
  if (nthr < 64) nthr = 64;
  if (nthr > 1024) nthr = 1024;
  const size_t lds = 2 * (size_t)N * sizeof(u32);
  auto kern = k_lds_conv<LN, LRA, 4, LAZY>;
  if (P.lq == 3) kern = k_lds_conv<LN, LRA, 3, LAZY>;
  hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<1, nthr, lds, s>>>(a, (int)la, b, (int)lb, c, (int)lc, P.ma, mp, T, sc, err);
  return hipGetLastError();
}

template <int LN, bool LAZY>
static hipError_t lds_conv_ra(const Plan& P, const u32* a, long la, const u32* b, long lb, u32* c, long lc,
                              const ModP& mp, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  switch (P.logRA) {
#define PM_RA(r)                                                                                  \
  case r:                                                                                         \
    if constexpr (r <= LN) return lds_conv_inst<LN, r, LAZY>(P, a, la, b, lb, c, lc, mp, T, sc, err, s); \
    break;
    PM_RA(1) PM_RA(2) PM_RA(3) PM_RA(4) PM_RA(5)
#undef PM_RA
    default:
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lds_conv(const Plan& P, const u32* a, long la, const u32* b, long lb, u32* c, long lc, int pidx,
                           const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_LN(n)                                                                          \
  case n:                                                                                 \
    return PI.lazy ? lds_conv_ra<n, true>(P, a, la, b, lb, c, lc, mp, T, sc, err, s)      \
                   : lds_conv_ra<n, false>(P, a, la, b, lb, c, lc, mp, T, sc, err, s);
  switch (P.logL) {
    PM_LN(6) PM_LN(7) PM_LN(8) PM_LN(9) PM_LN(10) PM_LN(11) PM_LN(12) PM_LN(13) PM_LN(14)
    default:
      break;
  }
#undef PM_LN
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// four-step column pass (forward), one sub-round (R = RA <= 32): one thread
// per column j2 loads x_{C j1 + j2}, j1 < RA (zero beyond the operand's
// length), transforms in registers and keeps output rows t < ma.
// blockIdx.y selects the operand.

template <int LRA, bool LAZY, typename TIn>
__global__ void __launch_bounds__(64) k_col_fwd1(const TIn* __restrict__ a, long za, const TIn* __restrict__ b, long zb,
                                                u32* __restrict__ Ta, u32* __restrict__ Tb, int logC, int ma, ModP mp,
                                                PrimeTables T, int* err) {
  constexpr int RA = 1 << LRA;
  const long C = 1l << logC;
  const long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j2 >= C) return;
  const Arith<LAZY> A(mp);
  const TIn* in = blockIdx.y ? b : a;
  const long z = blockIdx.y ? zb : za;
  u32* out = blockIdx.y ? Tb : Ta;
  u32 x[RA];
  bool bad = false;
#pragma unroll
  for (int s = 0; s < RA; ++s) {
    const long pos = C * s + j2;
    x[s] = pos < z ? (u32)in[pos] : 0u;
    bad |= x[s] >= mp.p;
  }
  if (bad) atomicOr(err, 1);
  dif_reg<RA>(A, x, T.pf);
#pragma unroll
  for (int t = 0; t < RA; ++t)
    if (t < ma) out[C * t + j2] = x[t];
}

// four-step column pass (forward), two sub-rounds (R = RA * RB): a work-group
// owns W adjacent columns.  Sub-round 1: thread (c, j1b) transforms rows
// j1b + RB e (e < RA) and twiddles by w_R^{j1b k1a}; sub-round 2: thread
// (c, ta) transforms the RB values of block ta, giving output row
// t = ta RB + tb.  Only blocks ta < ma are carried into sub-round 2.

template <int LRA, int LRB, int LW, bool LAZY, typename TIn>
__global__ void __launch_bounds__(1024) k_col_fwd2(const TIn* __restrict__ a, long za, const TIn* __restrict__ b,
                                                   long zb, u32* __restrict__ Ta, u32* __restrict__ Tb, int logC,
                                                   int ma, ModP mp, PrimeTables T, int* err) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, W = 1 << LW, R = RA * RB;
  extern __shared__ u32 sm[];  // [RA][RB][W]
  const long C = 1l << logC;
  const long c0 = (long)blockIdx.x * W;
  const Arith<LAZY> A(mp);
  const TIn* in = blockIdx.y ? b : a;
  const long z = blockIdx.y ? zb : za;
  u32* out = blockIdx.y ? Tb : Ta;
  const int tid = threadIdx.x, nthr = blockDim.x;
  bool bad = false;
  for (int task = tid; task < W * RB; task += nthr) {
    const int c = task & (W - 1);
    const int j1b = task >> LW;
    u32 x[RA];
#pragma unroll
    for (int e = 0; e < RA; ++e) {
      const long pos = C * (j1b + RB * e) + c0 + c;
      x[e] = pos < z ? (u32)in[pos] : 0u;
      bad |= x[e] >= mp.p;
    }
    dif_reg<RA>(A, x, T.pf);
#pragma unroll
    for (int ta = 0; ta < RA; ++ta) {
      if (ta < ma) {
        u32 v = x[ta];
        if (ta > 0 && j1b > 0) v = A.mul(v, T.pf[R + j1b * (int)(__brev((u32)ta) >> (32 - LRA))]);
        sm[(ta * RB + j1b) * W + c] = v;
      }
    }
  }
  if (bad) atomicOr(err, 1);
  __syncthreads();
  for (int task = tid; task < W * ma; task += nthr) {
    const int c = task & (W - 1);
    const int ta = task >> LW;
    u32 x[RB];
#pragma unroll
    for (int j1b = 0; j1b < RB; ++j1b) x[j1b] = sm[(ta * RB + j1b) * W + c];
    dif_reg<RB>(A, x, T.pf);
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) out[C * (ta * RB + tb) + c0 + c] = x[tb];
  }
}

template <int LRA, bool LAZY, typename TIn>
static hipError_t col_fwd_ra(const Plan& P, const TIn* a, long za, const TIn* b, long zb, u32* Ta, u32* Tb,
                             const ModP& mp, const PrimeTables& T, int* err, hipStream_t s) {
  const int nops = b ? 2 : 1;
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    dim3 grid((unsigned)((C + 63) / 64), (unsigned)nops);
    k_col_fwd1<LRA, LAZY, TIn><<<grid, 64, 0, s>>>(a, za, b, zb, Ta, Tb, P.logC, P.ma, mp, T, err);
    return hipGetLastError();
  }
  if constexpr (LRA == 5) {
    // W = 64 columns for RB <= 16, W = 32 for RB = 32 (LDS = R * W * 4 <= 128 KB)
    switch (P.logRB) {
#define PM_RB(rb, lw)                                                                                    \
  case rb: {                                                                                             \
    constexpr int W = 1 << lw;                                                                           \
    const size_t lds = (size_t)(32 << rb) * W * sizeof(u32);                                             \
    int nthr = W * ((1 << rb) > 32 ? (1 << rb) : 32);                                                     \
    if (nthr > 1024) nthr = 1024;                                                                        \
    auto kern = k_col_fwd2<5, rb, lw, LAZY, TIn>;                                                        \
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);        \
    dim3 grid((unsigned)(C / W), (unsigned)nops);                                                                     \
    kern<<<grid, nthr, lds, s>>>(a, za, b, zb, Ta, Tb, P.logC, P.ma, mp, T, err);                        \
    return hipGetLastError();                                                                            \
  }
      PM_RB(1, 6) PM_RB(2, 6) PM_RB(3, 6) PM_RB(4, 6) PM_RB(5, 5)
#undef PM_RB
      default:
        break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename TIn>
static hipError_t col_fwd_t(const Plan& P, const TIn* a, long za, const TIn* b, long zb, u32* Ta, u32* Tb, int pidx,
                            const PrimeTables& T, int* err, hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_RA(r)                                                                          \
  case r:                                                                                 \
    return PI.lazy ? col_fwd_ra<r, true, TIn>(P, a, za, b, zb, Ta, Tb, mp, T, err, s)      \
                   : col_fwd_ra<r, false, TIn>(P, a, za, b, zb, Ta, Tb, mp, T, err, s);
  switch (P.logRA) {
    PM_RA(1) PM_RA(2) PM_RA(3) PM_RA(4) PM_RA(5)
    default:
      break;
  }
#undef PM_RA
  return hipErrorInvalidValue;
}

hipError_t launch_col_fwd(const Plan& P, const void* a, long za, const void* b, long zb, int in_type, u32* Ta, u32* Tb,
                          int pidx, const PrimeTables& T, int* err, hipStream_t s) {
  if (in_type == 1)
    return col_fwd_t<uint16_t>(P, (const uint16_t*)a, za, (const uint16_t*)b, zb, Ta, Tb, pidx, T, err, s);
  return col_fwd_t<u32>(P, (const u32*)a, za, (const u32*)b, zb, Ta, Tb, pidx, T, err, s);
}

// ---------------------------------------------------------------------------
// four-step row pass of the convolution: row t (k1 = rev(t)) of both
// operands, twiddle by w_L^{j2 k1}, length-C transforms, pointwise product
// times the scale, inverse transform, untwiddle by w_L^{-j2 k1}.

template <int LC, int LQ, bool LAZY>
__global__ void __launch_bounds__(1024) k_row_conv(const u32* Ta, const u32* __restrict__ Tb, u32* Tc, int logR, ModP mp, PrimeTables T,
                                                   SplitTables S, uint2 sc) {
  constexpr int C = 1 << LC;
  extern __shared__ u32 sm[];
  u32* sa = sm;
  u32* sb = sm + C;
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int row = blockIdx.x;
  const u32 k1 = bitrev_n((u32)row, logR);
  const long off = (long)row * C;
  const u32 lomask = (1u << S.hbits) - 1u;
  for (int i = tid; i < C; i += nthr) {
    const u32 e = k1 * (u32)i;
    const uint2 w1 = S.lo_f[e & lomask];
    const uint2 w2 = S.hi_f[e >> S.hbits];
    sa[i] = A.mul(A.mul(Ta[off + i], w1), w2);
    sb[i] = A.mul(A.mul(Tb[off + i], w1), w2);
  }
  __syncthreads();
  u32* bufs[2] = {sa, sb};
  dif_lds<LC, LQ, LAZY, 2>(A, bufs, C, T.pf, tid, nthr);
  for (int i = tid; i < C; i += nthr) sa[i] = A.mul(A.mont(sa[i], sb[i]), sc);
  __syncthreads();
  dit_lds<LC, LQ, LAZY>(A, sa, C, T.pi, tid, nthr);
  for (int i = tid; i < C; i += nthr) {
    const u32 e = k1 * (u32)i;
    Tc[off + i] = A.mul(A.mul(sa[i], S.lo_i[e & lomask]), S.hi_i[e >> S.hbits]);
  }
}

template <int LC, bool LAZY>
static hipError_t row_conv_inst(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, const ModP& mp,
                                const PrimeTables& T, const SplitTables& S, uint2 sc, hipStream_t s) {
  constexpr int C = 1 << LC;
  const int rows = P.ma << P.logRB;
  const int logR = P.logRA + P.logRB;
  int nthr = C / 16;
  if (nthr > 1024) nthr = 1024;
  if (nthr < 64) nthr = 64;
  const size_t lds = 2 * (size_t)C * sizeof(u32);
  auto kern = P.lq == 3 ? k_row_conv<LC, 3, LAZY> : k_row_conv<LC, 4, LAZY>;
  hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<rows, nthr, lds, s>>>(Ta, Tb, Tc, logR, mp, T, S, sc);
  return hipGetLastError();
}

hipError_t launch_row_conv(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, int pidx, const PrimeTables& T,
                           const SplitTables& S, uint2 sc, hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_LC(n)                                                              \
  case n:                                                                     \
    return PI.lazy ? row_conv_inst<n, true>(P, Ta, Tb, Tc, mp, T, S, sc, s)   \
                   : row_conv_inst<n, false>(P, Ta, Tb, Tc, mp, T, S, sc, s);
  switch (P.logC) {
    PM_LC(10) PM_LC(11) PM_LC(12) PM_LC(13) PM_LC(14)
    default:
      break;
  }
#undef PM_LC
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// four-step column pass (inverse).  One sub-round: thread per column j2
// gathers rows t < ma, inverts (full length-RA inverse, or the truncated
// inverse with ma known values), writes coefficients j1 < ma.

template <int LRA, bool LAZY, typename TOut>
__global__ void __launch_bounds__(64) k_col_inv1(const u32* __restrict__ Tc, TOut* __restrict__ c, long lc, int logC,
                                                int ma, ModP mp, PrimeTables T) {
  constexpr int RA = 1 << LRA;
  const long C = 1l << logC;
  const long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j2 >= C) return;
  const Arith<LAZY> A(mp);
  u32 x[RA];
#pragma unroll
  for (int t = 0; t < RA; ++t) x[t] = t < ma ? Tc[C * t + j2] : 0u;
  inv_column<RA, LAZY>(A, x, ma, T);
#pragma unroll
  for (int s = 0; s < RA; ++s) {
    const long pos = C * s + j2;
    if (s < ma && pos < lc) c[pos] = (TOut)A.canon(x[s]);
  }
}

// two sub-rounds: inverse of k_col_fwd2
template <int LRA, int LRB, int LW, bool LAZY, typename TOut>
__global__ void __launch_bounds__(1024) k_col_inv2(const u32* __restrict__ Tc, TOut* __restrict__ c, long lc, int logC,
                                                   int ma, ModP mp, PrimeTables T) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, W = 1 << LW, R = RA * RB;
  extern __shared__ u32 sm[];  // [RA][RB][W]
  const long C = 1l << logC;
  const long c0 = (long)blockIdx.x * W;
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int task = tid; task < W * ma; task += nthr) {
    const int cc = task & (W - 1);
    const int ta = task >> LW;
    u32 x[RB];
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) x[tb] = Tc[C * (ta * RB + tb) + c0 + cc];
    dit_reg<RB>(A, x, T.pi);
#pragma unroll
    for (int j1b = 0; j1b < RB; ++j1b) sm[(ta * RB + j1b) * W + cc] = x[j1b];
  }
  __syncthreads();
  for (int task = tid; task < W * RB; task += nthr) {
    const int cc = task & (W - 1);
    const int j1b = task >> LW;
    u32 x[RA];
#pragma unroll
    for (int ta = 0; ta < RA; ++ta) {
      u32 v = 0;
      if (ta < ma) {
        v = sm[(ta * RB + j1b) * W + cc];
        if (ta > 0 && j1b > 0) v = A.mul(v, T.pi[R + j1b * (int)(__brev((u32)ta) >> (32 - LRA))]);
      }
      x[ta] = v;
    }
    inv_column<RA, LAZY>(A, x, ma, T);
#pragma unroll
    for (int e = 0; e < RA; ++e) {
      const long pos = C * (j1b + RB * e) + c0 + cc;
      if (e < ma && pos < lc) c[pos] = (TOut)A.canon(x[e]);
    }
  }
}

template <int LRA, bool LAZY>
static hipError_t col_inv_ra(const Plan& P, const u32* Tc, u32* c, long lc, const ModP& mp, const PrimeTables& T,
                             hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    k_col_inv1<LRA, LAZY, u32><<<(unsigned)((C + 63) / 64), 64, 0, s>>>(Tc, c, lc, P.logC, P.ma, mp, T);
    return hipGetLastError();
  }
  if constexpr (LRA == 5) {
    switch (P.logRB) {
#define PM_RB(rb, lw)                                                                             \
  case rb: {                                                                                      \
    constexpr int W = 1 << lw;                                                                    \
    const size_t lds = (size_t)(32 << rb) * W * sizeof(u32);                                      \
    int nthr = W * ((1 << rb) > 32 ? (1 << rb) : 32);                                              \
    if (nthr > 1024) nthr = 1024;                                                                 \
    auto kern = k_col_inv2<5, rb, lw, LAZY, u32>;                                                 \
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    kern<<<(unsigned)(C / W), nthr, lds, s>>>(Tc, c, lc, P.logC, P.ma, mp, T);                    \
    return hipGetLastError();                                                                     \
  }
      PM_RB(1, 6) PM_RB(2, 6) PM_RB(3, 6) PM_RB(4, 6) PM_RB(5, 5)
#undef PM_RB
      default:
        break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_col_inv(const Plan& P, const u32* Tc, u32* c, long lc, int pidx, const PrimeTables& T,
                          hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_RA(r)                                                           \
  case r:                                                                  \
    return PI.lazy ? col_inv_ra<r, true>(P, Tc, c, lc, mp, T, s)           \
                   : col_inv_ra<r, false>(P, Tc, c, lc, mp, T, s);
  switch (P.logRA) {
    PM_RA(1) PM_RA(2) PM_RA(3) PM_RA(4) PM_RA(5)
    default:
      break;
  }
#undef PM_RA
  return hipErrorInvalidValue;
}

}  // namespace pm
