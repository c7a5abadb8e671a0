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
// blockIdx.y selects the operand, blockIdx.z the job.

template <int LRA, bool LAZY, typename TIn>
__global__ void __launch_bounds__(64) k_col_fwd1(JobRef jr, int logC) {
  constexpr int RA = 1 << LRA;
  const ConvJob J = load_job(jr);
  const long C = 1l << logC;
  const long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j2 >= C) return;
  const Arith<LAZY> A(J.mp);
  const TIn* __restrict__ in = (const TIn*)(blockIdx.y ? J.b : J.a);
  const long z = blockIdx.y ? J.lb : J.la;
  u32* __restrict__ out = blockIdx.y ? J.Tb : J.Ta;
  u32 x[RA];
  bool bad = false;
#pragma unroll
  for (int s = 0; s < RA; ++s) {
    const long pos = C * s + j2;
    x[s] = pos < z ? (u32)in[pos] : 0u;
    bad |= x[s] >= J.mp.p;
  }
  if (bad) atomicOr(J.err, 1);
  dif_reg<RA>(A, x, J.T.pf);
#pragma unroll
  for (int t = 0; t < RA; ++t)
    if (t < J.ma) out[C * t + j2] = x[t];
}

// four-step column pass (forward), two sub-rounds (R = RA * RB): a work-group
// owns W adjacent columns.  Sub-round 1: thread (c, j1b) transforms rows
// j1b + RB e (e < RA) and twiddles by w_R^{j1b k1a}; sub-round 2: thread
// (c, ta) transforms the RB values of block ta, giving output row
// t = ta RB + tb.  Only blocks ta < ma are carried into sub-round 2.

template <int LRA, int LRB, int LW, bool LAZY, typename TIn>
__global__ void __launch_bounds__(1024) k_col_fwd2(JobRef jr, int logC) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, W = 1 << LW, R = RA * RB;
  extern __shared__ u32 sm[];  // [RA][RB][W]
  const ConvJob J = load_job(jr);
  const long C = 1l << logC;
  const long c0 = (long)blockIdx.x * W;
  const Arith<LAZY> A(J.mp);
  const TIn* __restrict__ in = (const TIn*)(blockIdx.y ? J.b : J.a);
  const long z = blockIdx.y ? J.lb : J.la;
  u32* __restrict__ out = blockIdx.y ? J.Tb : J.Ta;
  const int ma = J.ma;
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
      bad |= x[e] >= J.mp.p;
    }
    dif_reg<RA>(A, x, J.T.pf);
    uint2 tw[RA];
    load_tw<RA>(tw, J.T.rf[LRA - 1] + R + j1b * RA);
#pragma unroll
    for (int ta = 0; ta < RA; ++ta) {
      if (ta < ma) {
        u32 v = x[ta];
        if (ta > 0) v = A.mul(v, tw[ta]);
        sm[(ta * RB + j1b) * W + c] = v;
      }
    }
  }
  if (bad) atomicOr(J.err, 1);
  __syncthreads();
  for (int task = tid; task < W * ma; task += nthr) {
    const int c = task & (W - 1);
    const int ta = task >> LW;
    u32 x[RB];
#pragma unroll
    for (int j1b = 0; j1b < RB; ++j1b) x[j1b] = sm[(ta * RB + j1b) * W + c];
    dif_reg<RB>(A, x, J.T.pf);
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) out[C * (ta * RB + tb) + c0 + c] = x[tb];
  }
}

// Columns per work-group of the two-sub-round passes: W RB = 1024 first-
// round tasks (one per thread) unless the LDS tile W R words would exceed
// 64 KB, and at least 32 columns (128-byte row segments); at most 128 KB.
template <int LRA, int LRB>
constexpr int col_lw() {
  constexpr int a = 10 - LRB;
  constexpr int b = 14 - LRA - LRB;
  constexpr int w = a < b ? a : b;
  return w < 5 ? 5 : w;
}
template <int LRA, int LRB>
constexpr int col_threads() {
  constexpr int n = (1 << col_lw<LRA, LRB>()) << LRB;
  return n > 1024 ? 1024 : n;
}

template <int LRA, int LRB, typename TIn>
static hipError_t col_fwd2_launch(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  constexpr int LW = col_lw<LRA, LRB>();
  const long C = 1l << P.logC;
  if (C < (1l << LW)) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (LW + LRA + LRB)) * sizeof(u32);
  auto kern = k_col_fwd2<LRA, LRB, LW, kLazy, TIn>;
  ensure_lds_attr((const void*)kern, lds);
  TraceScope ts(s, "col_fwd");
  kern<<<dim3((unsigned)(C >> LW), nops, njobs), col_threads<LRA, LRB>(), lds, s>>>(jr, P.logC);
  return hipGetLastError();
}

template <int LRA, typename TIn>
static hipError_t col_fwd_ra(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    TraceScope ts(s, "col_fwd");
    k_col_fwd1<LRA, kLazy, TIn><<<dim3((unsigned)((C + 63) / 64), nops, njobs), 64, 0, s>>>(jr, P.logC);
    return hipGetLastError();
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_fwd2_launch<LRA, 1, TIn>(P, nops, jr, njobs, s);
      case 2: return col_fwd2_launch<LRA, 2, TIn>(P, nops, jr, njobs, s);
      case 3: return col_fwd2_launch<LRA, 3, TIn>(P, nops, jr, njobs, s);
      case 4: return col_fwd2_launch<LRA, 4, TIn>(P, nops, jr, njobs, s);
      case 5: return col_fwd2_launch<LRA, 5, TIn>(P, nops, jr, njobs, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename TIn>
static hipError_t col_fwd_t(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  switch (P.logRA) {
    case 1: return col_fwd_ra<1, TIn>(P, nops, jr, njobs, s);
    case 2: return col_fwd_ra<2, TIn>(P, nops, jr, njobs, s);
    case 3: return col_fwd_ra<3, TIn>(P, nops, jr, njobs, s);
    case 4: return col_fwd_ra<4, TIn>(P, nops, jr, njobs, s);
    case 5: return col_fwd_ra<5, TIn>(P, nops, jr, njobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_fwd)(const Plan& P, int in_type, int nops, const JobRef& jr, int njobs,
                                     hipStream_t s) {
  if (in_type == 1) return col_fwd_t<uint16_t>(P, nops, jr, njobs, s);
  return col_fwd_t<u32>(P, nops, jr, njobs, s);
}

// ---------------------------------------------------------------------------
// four-step row pass of the convolution: row t (k1 = rev(t)) of both
// operands, twiddle by w_L^{j2 k1}, length-C transforms, pointwise product,
// inverse transform, untwiddle by w_L^{-j2 k1} times the scale (which also
// undoes the Montgomery factor of the product).  The result overwrites Ta.
//
// Thread tid loads elements tid + NT e (coalesced), so its EPT = C / NT
// values are exactly one group of the outermost radix-EPT round: that round
// runs in registers straight after the load, and its inverse straight before
// the store.  The innermost round (contiguous groups) also stays in
// registers, so the product is formed and inverted there without a trip
// through LDS.  Only the rounds between cross LDS.  NB = 2 keeps both operands
// in LDS at once so their rounds share barriers; NB = 1 (the largest rows)
// transforms them one after the other in one buffer.

template <int LC, int LE, bool LAZY>
__device__ __forceinline__ void row_twist_fwd(const Arith<LAZY>& A, u32 (&x)[1 << LE], uint2 g,
                                              const uint2* __restrict__ f, const PrimeTables& T, int tid) {
#pragma unroll
  for (int e = 0; e < (1 << LE); ++e) x[e] = A.mul(A.mul(x[e], g), f[e]);
  dif_top_reg<LC, LE, LAZY>(A, x, T, tid);
}

template <int LQL, int EPT, bool LAZY>
__device__ __forceinline__ void row_last_fwd(const Arith<LAZY>& A, const u32* buf, u32 (&x)[EPT],
                                             const PrimeTables& T, int tid, int nthr) {
  constexpr int QL = 1 << LQL;
#pragma unroll
  for (int u = 0; u < EPT / QL; ++u) {
    u32 y[QL];
    lds_load_contig<QL>(buf, (tid + nthr * u) * QL, y);
    dif_reg<QL>(A, y, T.pf);
#pragma unroll
    for (int t = 0; t < QL; ++t) x[u * QL + t] = y[t];
  }
}

template <int LC, int LQ, int LNT, int NB, bool LAZY>
__global__ void __launch_bounds__(1 << LNT) k_row_conv(JobRef jr, int logR) {
  constexpr int C = 1 << LC;
  constexpr int NT = 1 << LNT;
  constexpr int LE = LC - LNT;
  constexpr int EPT = 1 << LE;
  constexpr int LQL = last_lb<LNT, LQ>();
  constexpr int QL = 1 << LQL;
  static_assert(QL <= EPT, "innermost round wider than a thread's share");
  const ConvJob J = load_job(jr);
  const int row = blockIdx.x;
  if (row >= J.rows) return;
  extern __shared__ u32 sm[];
  u32* const sa = sm;
  u32* const sb = sm + (NB - 1) * C;
  const Arith<LAZY> A(J.mp);
  const int tid = threadIdx.x;
  const u32 k1 = bitrev_n((u32)row, logR);
  const long off = (long)row * C;
  u32* Ta = J.Ta;
  const u32* __restrict__ Tb = J.Tb;
  const uint2 gf = J.W.gf[k1 * (u32)tid];
  const uint2* ff = J.W.ff + (size_t)k1 * EPT;
  // b's row is fetched up front (its latency hides behind a's rounds) unless
  // 1024 threads leave too few registers to hold it meanwhile
  constexpr bool kPrefetchB = NB == 2 || LNT < 10;
  u32 xa[EPT], xb[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    xa[e] = Ta[off + tid + NT * e];
    if constexpr (kPrefetchB) xb[e] = Tb[off + tid + NT * e];
  }
  row_twist_fwd<LC, LE, LAZY>(A, xa, gf, ff, J.T, tid);
#pragma unroll
  for (int t = 0; t < EPT; ++t) sa[lds_ix(tid + NT * t)] = xa[t];
  if constexpr (NB == 2) {
    row_twist_fwd<LC, LE, LAZY>(A, xb, gf, ff, J.T, tid);
#pragma unroll
    for (int t = 0; t < EPT; ++t) sb[lds_ix(tid + NT * t)] = xb[t];
  }
  __syncthreads();
  if constexpr (NB == 2) {
    u32* bufs[2] = {sa, sb};
    dif_lds_upto<LNT, LQL, LQ, LAZY, 2>(A, bufs, C, J.T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xa, J.T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sb, xb, J.T, tid, NT);
  } else {
    u32* bufs[1] = {sa};
    dif_lds_upto<LNT, LQL, LQ, LAZY, 1>(A, bufs, C, J.T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xa, J.T, tid, NT);
    if constexpr (!kPrefetchB) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) xb[e] = Tb[off + tid + NT * e];
    }
    __syncthreads();
    row_twist_fwd<LC, LE, LAZY>(A, xb, gf, ff, J.T, tid);
#pragma unroll
    for (int t = 0; t < EPT; ++t) sa[lds_ix(tid + NT * t)] = xb[t];
    __syncthreads();
    dif_lds_upto<LNT, LQL, LQ, LAZY, 1>(A, bufs, C, J.T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xb, J.T, tid, NT);
  }
  // pointwise product and the innermost inverse round; each thread writes
  // back exactly the LDS words it read last, so no barrier is needed first
#pragma unroll
  for (int u = 0; u < EPT / QL; ++u) {
    u32 y[QL];
#pragma unroll
    for (int t = 0; t < QL; ++t) y[t] = A.mont(xa[u * QL + t], xb[u * QL + t]);
    dit_reg<QL>(A, y, J.T.pi);
    lds_store_contig<QL>(sa, (tid + NT * u) * QL, y);
  }
  __syncthreads();
  dit_lds_from<LNT, LQL, LQ, LAZY>(A, sa, C, J.T, tid, NT);
#pragma unroll
  for (int t = 0; t < EPT; ++t) xa[t] = sa[lds_ix(tid + NT * t)];
  dit_top_reg<LC, LE, LAZY>(A, xa, J.T, tid);
  const uint2 gi = J.W.gi[k1 * (u32)tid];
  const uint2* fi = J.W.fi + (size_t)k1 * EPT;
#pragma unroll
  for (int e = 0; e < EPT; ++e) Ta[off + tid + NT * e] = A.mul(A.mul(xa[e], gi), fi[e]);
}

template <int LC, int LNT>
static hipError_t row_conv_inst(const Plan& P, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  constexpr int C = 1 << LC;
  constexpr int NB = LC <= 13 ? 2 : 1;
  const int logR = P.logRA + P.logRB;
  const size_t lds = (size_t)NB * C * sizeof(u32);
  auto kern = P.lq == 3 ? k_row_conv<LC, 3, LNT, NB, kLazy> : k_row_conv<LC, 4, LNT, NB, kLazy>;
  ensure_lds_attr((const void*)kern, lds);
  TraceScope ts(s, "row_conv");
  kern<<<dim3(max_rows, 1, njobs), 1 << LNT, lds, s>>>(jr, logR);
  return hipGetLastError();
}

template <int LC>
static hipError_t row_conv_lc(const Plan& P, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  switch (plan_row_lnt(P)) {
#define PM_NT(n)                                                               \
  case n:                                                                      \
    if constexpr (LC - n >= 4 && LC - n <= 6 && n >= 6 && n <= 10)             \
      return row_conv_inst<LC, n>(P, max_rows, jr, njobs, s);                  \
    break;
    PM_NT(6) PM_NT(7) PM_NT(8) PM_NT(9) PM_NT(10)
#undef PM_NT
    default:
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_row_conv)(const Plan& P, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  switch (P.logC) {
    case 10: return row_conv_lc<10>(P, max_rows, jr, njobs, s);
    case 11: return row_conv_lc<11>(P, max_rows, jr, njobs, s);
    case 12: return row_conv_lc<12>(P, max_rows, jr, njobs, s);
    case 13: return row_conv_lc<13>(P, max_rows, jr, njobs, s);
    case 14: return row_conv_lc<14>(P, max_rows, jr, njobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// four-step column pass (inverse), reading Ta.  One sub-round: thread per
// column j2 gathers rows t < ma, inverts (full length-RA inverse, or the
// truncated inverse with ma known values), writes coefficients j1 < ma.

template <int LRA, bool LAZY>
__global__ void __launch_bounds__(64) k_col_inv1(JobRef jr, int logC) {
  constexpr int RA = 1 << LRA;
  const ConvJob J = load_job(jr);
  const long C = 1l << logC;
  const long j2 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j2 >= C) return;
  const Arith<LAZY> A(J.mp);
  const u32* __restrict__ Tc = J.Ta;
  u32* __restrict__ c = J.c;
  const int ma = J.ma;
  u32 x[RA];
#pragma unroll
  for (int t = 0; t < RA; ++t) x[t] = t < ma ? Tc[C * t + j2] : 0u;
  inv_column<RA, LAZY>(A, x, ma, J.T);
#pragma unroll
  for (int s = 0; s < RA; ++s) {
    const long pos = C * s + j2;
    if (s < ma && pos < J.lc) c[pos] = A.canon(x[s]);
  }
}

// two sub-rounds: inverse of k_col_fwd2
template <int LRA, int LRB, int LW, bool LAZY>
__global__ void __launch_bounds__(1024) k_col_inv2(JobRef jr, int logC) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, W = 1 << LW, R = RA * RB;
  extern __shared__ u32 sm[];  // [RA][RB][W]
  const ConvJob J = load_job(jr);
  const long C = 1l << logC;
  const long c0 = (long)blockIdx.x * W;
  const Arith<LAZY> A(J.mp);
  const u32* __restrict__ Tc = J.Ta;
  u32* __restrict__ c = J.c;
  const int ma = J.ma;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int task = tid; task < W * ma; task += nthr) {
    const int cc = task & (W - 1);
    const int ta = task >> LW;
    u32 x[RB];
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) x[tb] = Tc[C * (ta * RB + tb) + c0 + cc];
    dit_reg<RB>(A, x, J.T.pi);
#pragma unroll
    for (int j1b = 0; j1b < RB; ++j1b) sm[(ta * RB + j1b) * W + cc] = x[j1b];
  }
  __syncthreads();
  for (int task = tid; task < W * RB; task += nthr) {
    const int cc = task & (W - 1);
    const int j1b = task >> LW;
    uint2 tw[RA];
    load_tw<RA>(tw, J.T.ri[LRA - 1] + R + j1b * RA);
    u32 x[RA];
#pragma unroll
    for (int ta = 0; ta < RA; ++ta) {
      u32 v = 0;
      if (ta < ma) {
        v = sm[(ta * RB + j1b) * W + cc];
        if (ta > 0) v = A.mul(v, tw[ta]);
      }
      x[ta] = v;
    }
    inv_column<RA, LAZY>(A, x, ma, J.T);
#pragma unroll
    for (int e = 0; e < RA; ++e) {
      const long pos = C * (j1b + RB * e) + c0 + cc;
      if (e < ma && pos < J.lc) c[pos] = A.canon(x[e]);
    }
  }
}

template <int LRA, int LRB>
static hipError_t col_inv2_launch(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  constexpr int LW = col_lw<LRA, LRB>();
  const long C = 1l << P.logC;
  if (C < (1l << LW)) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (LW + LRA + LRB)) * sizeof(u32);
  auto kern = k_col_inv2<LRA, LRB, LW, kLazy>;
  ensure_lds_attr((const void*)kern, lds);
  TraceScope ts(s, "col_inv");
  kern<<<dim3((unsigned)(C >> LW), 1, njobs), col_threads<LRA, LRB>(), lds, s>>>(jr, P.logC);
  return hipGetLastError();
}

template <int LRA>
static hipError_t col_inv_ra(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    TraceScope ts(s, "col_inv");
    k_col_inv1<LRA, kLazy><<<dim3((unsigned)((C + 63) / 64), 1, njobs), 64, 0, s>>>(jr, P.logC);
    return hipGetLastError();
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_inv2_launch<LRA, 1>(P, jr, njobs, s);
      case 2: return col_inv2_launch<LRA, 2>(P, jr, njobs, s);
      case 3: return col_inv2_launch<LRA, 3>(P, jr, njobs, s);
      case 4: return col_inv2_launch<LRA, 4>(P, jr, njobs, s);
      case 5: return col_inv2_launch<LRA, 5>(P, jr, njobs, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_inv)(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  switch (P.logRA) {
    case 1: return col_inv_ra<1>(P, jr, njobs, s);
    case 2: return col_inv_ra<2>(P, jr, njobs, s);
    case 3: return col_inv_ra<3>(P, jr, njobs, s);
    case 4: return col_inv_ra<4>(P, jr, njobs, s);
    case 5: return col_inv_ra<5>(P, jr, njobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace pm
