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
#ifndef PM_LAZY
#error "compile with -DPM_LAZY=0 or -DPM_LAZY=1"
#endif
#define PM_CAT2(a, b) a##b
#define PM_CAT(a, b) PM_CAT2(a, b)
#define PM_SUFFIX(name) PM_CAT(name, PM_CAT(_lazy, PM_LAZY))
#include "internal.h"
#include "trace.h"

namespace pm {
constexpr bool kLazy = PM_LAZY != 0;

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
        if (ta > 0 && j1b > 0) v = A.mul(v, T.rf[LRA - 3][R + j1b * RA + ta]);
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

// columns per work-group of the two-sub-round passes: 64 for R <= 2^8,
// else 32 (LDS = R * W * 4 bytes, at most 128 KB)
template <int LR>
constexpr int col_lw() {
  return LR <= 8 ? 6 : 5;
}

template <int LRA, int LRB, bool LAZY, typename TIn>
static hipError_t col_fwd2_launch(const Plan& P, const TIn* a, long za, const TIn* b, long zb, u32* Ta, u32* Tb,
                                  int nops, const ModP& mp, const PrimeTables& T, int* err, hipStream_t s) {
  constexpr int LW = col_lw<LRA + LRB>();
  constexpr int W = 1 << LW;
  const long C = 1l << P.logC;
  const size_t lds = ((size_t)W << (LRA + LRB)) * sizeof(u32);
  int nthr = W * ((1 << LRB) > (1 << LRA) ? (1 << LRB) : (1 << LRA));
  if (nthr > 1024) nthr = 1024;
  auto kern = k_col_fwd2<LRA, LRB, LW, LAZY, TIn>;
  (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  dim3 grid((unsigned)(C / W), (unsigned)nops);
  TraceScope ts(s, "col_fwd");
  kern<<<grid, nthr, lds, s>>>(a, za, b, zb, Ta, Tb, P.logC, P.ma, mp, T, err);
  return hipGetLastError();
}

template <int LRA, bool LAZY, typename TIn>
static hipError_t col_fwd_ra(const Plan& P, const TIn* a, long za, const TIn* b, long zb, u32* Ta, u32* Tb,
                             const ModP& mp, const PrimeTables& T, int* err, hipStream_t s) {
  const int nops = b ? 2 : 1;
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    dim3 grid((unsigned)((C + 63) / 64), (unsigned)nops);
    TraceScope ts(s, "col_fwd");
    k_col_fwd1<LRA, LAZY, TIn><<<grid, 64, 0, s>>>(a, za, b, zb, Ta, Tb, P.logC, P.ma, mp, T, err);
    return hipGetLastError();
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_fwd2_launch<LRA, 1, LAZY, TIn>(P, a, za, b, zb, Ta, Tb, nops, mp, T, err, s);
      case 2: return col_fwd2_launch<LRA, 2, LAZY, TIn>(P, a, za, b, zb, Ta, Tb, nops, mp, T, err, s);
      case 3: return col_fwd2_launch<LRA, 3, LAZY, TIn>(P, a, za, b, zb, Ta, Tb, nops, mp, T, err, s);
      case 4: return col_fwd2_launch<LRA, 4, LAZY, TIn>(P, a, za, b, zb, Ta, Tb, nops, mp, T, err, s);
      case 5: return col_fwd2_launch<LRA, 5, LAZY, TIn>(P, a, za, b, zb, Ta, Tb, nops, mp, T, err, s);
      default: break;
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
    return col_fwd_ra<r, kLazy, TIn>(P, a, za, b, zb, Ta, Tb, mp, T, err, s);
  switch (P.logRA) {
    PM_RA(1) PM_RA(2) PM_RA(3) PM_RA(4) PM_RA(5)
    default:
      break;
  }
#undef PM_RA
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_fwd)(const Plan& P, const void* a, long za, const void* b, long zb, int in_type, u32* Ta, u32* Tb,
                          int pidx, const PrimeTables& T, int* err, hipStream_t s) {
  if (in_type == 1)
    return col_fwd_t<uint16_t>(P, (const uint16_t*)a, za, (const uint16_t*)b, zb, Ta, Tb, pidx, T, err, s);
  return col_fwd_t<u32>(P, (const u32*)a, za, (const u32*)b, zb, Ta, Tb, pidx, T, err, s);
}

// ---------------------------------------------------------------------------
// four-step row pass of the convolution: row t (k1 = rev(t)) of both
// operands, twiddle by w_L^{j2 k1}, length-C transforms, pointwise product,
// inverse transform, untwiddle by w_L^{-j2 k1} times the scale (which also
// undoes the Montgomery factor of the product).  One LDS buffer: the last
// forward round of each operand and the first inverse round stay in
// registers, so the product never goes back to LDS between the transforms.

template <int LC, int LQ, int LNT, bool LAZY>
__global__ void __launch_bounds__(1 << LNT) k_row_conv(const u32* Ta, const u32* __restrict__ Tb, u32* Tc, int logR,
                                                       ModP mp, PrimeTables T, RowTables W) {
  constexpr int C = 1 << LC;
  constexpr int NT = 1 << LNT;
  constexpr int EPT = C / NT;
  extern __shared__ u32 sm[];
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x;
  const int row = blockIdx.x;
  const u32 k1 = bitrev_n((u32)row, logR);
  const long off = (long)row * C;
  const uint2 gf = W.gf[k1 * (u32)tid];
  const uint2 gi = W.gi[k1 * (u32)tid];
  const uint2* ff = W.ff + (size_t)k1 * EPT;
  const uint2* fi = W.fi + (size_t)k1 * EPT;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = tid + NT * e;
    sm[lds_ix(i)] = A.mul(A.mul(Ta[off + i], gf), ff[e]);
  }
  __syncthreads();
  u32 xa[EPT];
  dif_lds_to_regs<LC, LQ, LAZY, EPT>(A, sm, C, T, tid, NT, xa);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = tid + NT * e;
    sm[lds_ix(i)] = A.mul(A.mul(Tb[off + i], gf), ff[e]);
  }
  __syncthreads();
  u32 xb[EPT];
  dif_lds_to_regs<LC, LQ, LAZY, EPT>(A, sm, C, T, tid, NT, xb);
#pragma unroll
  for (int e = 0; e < EPT; ++e) xa[e] = A.mont(xa[e], xb[e]);
  __syncthreads();
  dit_regs_to_lds<LC, LQ, LAZY, EPT>(A, sm, C, T, tid, NT, xa);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = tid + NT * e;
    Tc[off + i] = A.mul(A.mul(sm[lds_ix(i)], gi), fi[e]);
  }
}

template <int LC, int LNT, bool LAZY>
static hipError_t row_conv_inst(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, const ModP& mp,
                                const PrimeTables& T, const RowTables& W, hipStream_t s) {
  constexpr int C = 1 << LC;
  const int rows = P.ma << P.logRB;
  const int logR = P.logRA + P.logRB;
  const size_t lds = (size_t)C * sizeof(u32);
  auto kern = P.lq == 3 ? k_row_conv<LC, 3, LNT, LAZY> : k_row_conv<LC, 4, LNT, LAZY>;
  (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  TraceScope ts(s, "row_conv");
  kern<<<rows, 1 << LNT, lds, s>>>(Ta, Tb, Tc, logR, mp, T, W);
  return hipGetLastError();
}

template <int LC>
static hipError_t row_conv_lc(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, const ModP& mp,
                              const PrimeTables& T, const RowTables& W, hipStream_t s) {
  // 16 to 64 elements per thread, 64 to 1024 threads
  switch (plan_row_lnt(P)) {
#define PM_NT(n)                                                                                  \
  case n:                                                                                         \
    if constexpr (LC - n >= 4 && LC - n <= 6 && n >= 6 && n <= 10)                                \
      return row_conv_inst<LC, n, kLazy>(P, Ta, Tb, Tc, mp, T, W, s);                             \
    break;
    PM_NT(6) PM_NT(7) PM_NT(8) PM_NT(9) PM_NT(10)
#undef PM_NT
    default:
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_row_conv)(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, int pidx,
                                      const PrimeTables& T, const RowTables& W, hipStream_t s) {
  const ModP mp = modp_of(prime_info(pidx));
  switch (P.logC) {
#define PM_LC(n) \
  case n:        \
    return row_conv_lc<n>(P, Ta, Tb, Tc, mp, T, W, s);
    PM_LC(10) PM_LC(11) PM_LC(12) PM_LC(13) PM_LC(14)
#undef PM_LC
    default:
      break;
  }
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
        if (ta > 0 && j1b > 0) v = A.mul(v, T.ri[LRA - 3][R + j1b * RA + ta]);
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

template <int LRA, int LRB, bool LAZY>
static hipError_t col_inv2_launch(const Plan& P, const u32* Tc, u32* c, long lc, const ModP& mp,
                                  const PrimeTables& T, hipStream_t s) {
  constexpr int LW = col_lw<LRA + LRB>();
  constexpr int W = 1 << LW;
  const long C = 1l << P.logC;
  const size_t lds = ((size_t)W << (LRA + LRB)) * sizeof(u32);
  int nthr = W * ((1 << LRB) > (1 << LRA) ? (1 << LRB) : (1 << LRA));
  if (nthr > 1024) nthr = 1024;
  auto kern = k_col_inv2<LRA, LRB, LW, LAZY, u32>;
  (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  TraceScope ts(s, "col_inv");
  kern<<<(unsigned)(C / W), nthr, lds, s>>>(Tc, c, lc, P.logC, P.ma, mp, T);
  return hipGetLastError();
}

template <int LRA, bool LAZY>
static hipError_t col_inv_ra(const Plan& P, const u32* Tc, u32* c, long lc, const ModP& mp, const PrimeTables& T,
                             hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    TraceScope ts(s, "col_inv");
    k_col_inv1<LRA, LAZY, u32><<<(unsigned)((C + 63) / 64), 64, 0, s>>>(Tc, c, lc, P.logC, P.ma, mp, T);
    return hipGetLastError();
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_inv2_launch<LRA, 1, LAZY>(P, Tc, c, lc, mp, T, s);
      case 2: return col_inv2_launch<LRA, 2, LAZY>(P, Tc, c, lc, mp, T, s);
      case 3: return col_inv2_launch<LRA, 3, LAZY>(P, Tc, c, lc, mp, T, s);
      case 4: return col_inv2_launch<LRA, 4, LAZY>(P, Tc, c, lc, mp, T, s);
      case 5: return col_inv2_launch<LRA, 5, LAZY>(P, Tc, c, lc, mp, T, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_inv)(const Plan& P, const u32* Tc, u32* c, long lc, int pidx, const PrimeTables& T,
                          hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_RA(r)                                                           \
  case r:                                                                  \
    return col_inv_ra<r, kLazy>(P, Tc, c, lc, mp, T, s);
  switch (P.logRA) {
    PM_RA(1) PM_RA(2) PM_RA(3) PM_RA(4) PM_RA(5)
    default:
      break;
  }
#undef PM_RA
  return hipErrorInvalidValue;
}

}  // namespace pm
