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
#include "colpass.h"
#include "internal.h"
#include "trace.h"

namespace pm {

constexpr bool kLazy = PM_LAZY != 0;

// ---------------------------------------------------------------------------
// four-step column pass (forward), one sub-round (R = RA <= 32): one thread
// per column j2 loads x_{C j1 + j2}, j1 < RA (zero beyond the operand's
// length), transforms in registers and keeps output rows t < ma.
// blockIdx.y selects the operand, blockIdx.z the job.

template <int LRA, bool LAZY, typename TIn, bool TWIST>
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
    x[s] = pos < z ? (u32)gld(in + pos) : 0u;
    bad |= x[s] >= J.mp.p;
    if constexpr (TWIST) x[s] = A.mul(x[s], cld(J.twf + s));
  }
  if (bad) atomicOr(J.err, 1);
  if ((C << (LRA - 1)) >= z)  // rows RA/2 and up are zero
    dif_reg<RA, LAZY, false, true>(A, x, J.T.pf);
  else
    dif_reg<RA>(A, x, J.T.pf);
#pragma unroll
  for (int t = 0; t < RA; ++t)
    if (t < J.ma) gst(out + C * t + j2, x[t]);
}

// ---------------------------------------------------------------------------
// four-step column passes for R = RA RB > 32 rows.  A work-group of
// NT = W R / 16 threads owns W adjacent columns (an [R][W] LDS tile) and runs
// their length-R transforms as rounds of radix 2^LQ <= 16, each thread taking
// 16 / 2^LQ (column, group) tasks per round, lanes along the columns: so
// every thread holds 16 values per round, and the first round (straight
// from global memory) has 16 loads per thread in flight.  The last round
// writes global memory.  Only rows below mr = ma RB are kept (the relaxed
// TFT): blocks that start at or beyond mr are skipped.

template <int LR, bool LAZY, typename TIn, bool TWIST>
__global__ void __launch_bounds__(1024) k_col_fwdr(JobRef jr, int logC, int lw) {
  extern __shared__ u32 sm[];  // [R][W]
  const ConvJob J = load_job(jr);
  const Arith<LAZY> A(J.mp);
  const TIn* __restrict__ in = (const TIn*)(blockIdx.y ? J.b : J.a);
  const long z = blockIdx.y ? J.lb : J.la;
  u32* __restrict__ out = blockIdx.y ? J.Tb : J.Ta;
  bool bad = false;
  col_dif_rounds<LR, 0, LR, LAZY, TIn, TWIST>(A, sm, lw, J.rows, J.T, threadIdx.x, blockDim.x, in, z, 1l << logC,
                                       (long)blockIdx.x << lw, out, J.twf, bad);
  if (bad) atomicOr(J.err, 1);
}

template <int LR, typename TIn, bool TWIST>
static hipError_t col_fwdr_launch(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  const long groups = (long)nops * njobs;
  const int lw = col_lw(LR, P.logC, groups, groups == 1 ? 512 : 256);
  const long C = 1l << P.logC;
  if (C < (1l << lw) || col_threads(LR, lw) > 1024) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (lw + LR)) * sizeof(u32);
  auto kern = k_col_fwdr<LR, kLazy, TIn, TWIST>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("col_fwd", kern, dim3((unsigned)(C >> lw), nops, njobs), col_threads(LR, lw), lds, s, jr, P.logC,
                lw);
}

template <int LRA, typename TIn, bool TWIST>
static hipError_t col_fwd_ra(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    return launch("col_fwd", k_col_fwd1<LRA, kLazy, TIn, TWIST>, dim3((unsigned)((C + 63) / 64), nops, njobs), 64, 0,
                  s, jr, P.logC);
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_fwdr_launch<LRA + 1, TIn, TWIST>(P, nops, jr, njobs, s);
      case 2: return col_fwdr_launch<LRA + 2, TIn, TWIST>(P, nops, jr, njobs, s);
      case 3: return col_fwdr_launch<LRA + 3, TIn, TWIST>(P, nops, jr, njobs, s);
      case 4: return col_fwdr_launch<LRA + 4, TIn, TWIST>(P, nops, jr, njobs, s);
      case 5: return col_fwdr_launch<LRA + 5, TIn, TWIST>(P, nops, jr, njobs, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename TIn, bool TWIST>
static hipError_t col_fwd_t(const Plan& P, int nops, const JobRef& jr, int njobs, hipStream_t s) {
  switch (P.logRA) {
    case 1: return col_fwd_ra<1, TIn, TWIST>(P, nops, jr, njobs, s);
    case 2: return col_fwd_ra<2, TIn, TWIST>(P, nops, jr, njobs, s);
    case 3: return col_fwd_ra<3, TIn, TWIST>(P, nops, jr, njobs, s);
    case 4: return col_fwd_ra<4, TIn, TWIST>(P, nops, jr, njobs, s);
    case 5: return col_fwd_ra<5, TIn, TWIST>(P, nops, jr, njobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_fwd)(const Plan& P, int in_type, int nops, const JobRef& jr, int njobs,
                                     hipStream_t s) {
  if (in_type == 1) return P.twist ? hipErrorInvalidValue : col_fwd_t<uint16_t, false>(P, nops, jr, njobs, s);
  if (P.twist) return col_fwd_t<u32, true>(P, nops, jr, njobs, s);
  return col_fwd_t<u32, false>(P, nops, jr, njobs, s);
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
  const uint2 gf = cld(J.W.gf + k1 * (u32)NT + tid);
  const uint2* ff = J.W.ff + (size_t)k1 * EPT;
  // b's row is fetched up front (its latency hides behind a's rounds) unless
  // 1024 threads leave too few registers to hold it meanwhile
  constexpr bool kPrefetchB = NB == 2;
  PrimeTables T = J.T;
  u32 xa[EPT], xb[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    xa[e] = gld(Ta + off + tid + NT * e);
    if constexpr (kPrefetchB) xb[e] = gld(Tb + off + tid + NT * e);
  }
  row_twist_fwd<LC, LE, LAZY>(A, xa, gf, ff, T, tid);
#pragma unroll
  for (int t = 0; t < EPT; ++t) sa[lds_ix(tid + NT * t)] = xa[t];
  if constexpr (NB == 2) {
    row_twist_fwd<LC, LE, LAZY>(A, xb, gf, ff, T, tid);
#pragma unroll
    for (int t = 0; t < EPT; ++t) sb[lds_ix(tid + NT * t)] = xb[t];
  }
  __syncthreads();
  if constexpr (NB == 2) {
    u32* bufs[2] = {sa, sb};
    dif_lds_upto<LNT, LQL, LQ, LAZY, 2>(A, bufs, C, T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xa, T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sb, xb, T, tid, NT);
  } else {
    u32* bufs[1] = {sa};
    dif_lds_upto<LNT, LQL, LQ, LAZY, 1>(A, bufs, C, T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xa, T, tid, NT);
    T = fresh(T);
    ff = fresh(ff);
    if constexpr (!kPrefetchB) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) xb[e] = gld(Tb + off + tid + NT * e);
    }
    __syncthreads();
    row_twist_fwd<LC, LE, LAZY>(A, xb, gf, ff, T, tid);
#pragma unroll
    for (int t = 0; t < EPT; ++t) sa[lds_ix(tid + NT * t)] = xb[t];
    __syncthreads();
    dif_lds_upto<LNT, LQL, LQ, LAZY, 1>(A, bufs, C, T, tid, NT);
    row_last_fwd<LQL, EPT, LAZY>(A, sa, xb, T, tid, NT);
  }
  T = fresh(T);
  // pointwise product and the innermost inverse round; each thread writes
  // back exactly the LDS words it read last, so no barrier is needed first
#pragma unroll
  for (int u = 0; u < EPT / QL; ++u) {
    u32 y[QL];
#pragma unroll
    for (int t = 0; t < QL; ++t) y[t] = A.mont(xa[u * QL + t], xb[u * QL + t]);
    dit_reg<QL>(A, y, T.pi);
    lds_store_contig<QL>(sa, (tid + NT * u) * QL, y);
  }
  __syncthreads();
  dit_lds_from<LNT, LQL, LQ, LAZY>(A, sa, C, T, tid, NT);
#pragma unroll
  for (int t = 0; t < EPT; ++t) xa[t] = sa[lds_ix(tid + NT * t)];
  dit_top_reg<LC, LE, LAZY>(A, xa, T, tid);
  const uint2 gi = cld(J.W.gi + k1 * (u32)NT + tid);
  const uint2* fi = J.W.fi + (size_t)k1 * EPT;
#pragma unroll
  for (int e = 0; e < EPT; ++e) gst(Ta + off + tid + NT * e, A.mul(A.mul_raw(xa[e], gi), cld(fi + e)));
}

template <int LC, int LNT>
static hipError_t row_conv_inst(const Plan& P, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  constexpr int C = 1 << LC;
  constexpr int NB = LC <= 13 ? 2 : 1;
  const int logR = P.logRA + P.logRB;
  const size_t lds = (size_t)NB * C * sizeof(u32);
  auto kern = k_row_conv<LC, 3, LNT, NB, kLazy>;
  if constexpr (LC - LNT >= 4) {
    if (P.lq == 4) kern = k_row_conv<LC, 4, LNT, NB, kLazy>;
  }
  ensure_lds_attr((const void*)kern, lds);
  return launch("row_conv", kern, dim3(max_rows, 1, njobs), 1 << LNT, lds, s, jr, logR);
}

template <int LC>
static hipError_t row_conv_lc(const Plan& P, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  switch (plan_row_lnt(P)) {
#define PM_NT(n)                                                               \
  case n:                                                                      \
    if constexpr (LC - n >= 3 && LC - n <= 5 && n >= 6 && n <= 10)             \
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

template <int LRA, bool LAZY, bool TWIST>
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
  for (int t = 0; t < RA; ++t) x[t] = t < ma ? gld(Tc + C * t + j2) : 0u;
  inv_column<RA, LAZY>(A, x, ma, J.T);
#pragma unroll
  for (int s = 0; s < RA; ++s) {
    const long pos = C * s + j2;
    if (s < ma && pos < J.lc) gst(c + pos, A.canon(TWIST ? A.mul(x[s], cld(J.twi + s)) : x[s]));
  }
}

// Inverse column pass: the length-RB inverses of the blocks below mr (the
// innermost round straight from global memory), then per column and j1b
// the truncated inverse of radix RA with ma known values, written to the
// output coefficients.
template <int LRA, int LRB, bool LAZY, bool TWIST>
__global__ void __launch_bounds__(1024) k_col_invr(JobRef jr, int logC, int lw) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, R = RA * RB;
  extern __shared__ u32 sm[];  // [R][W]
  const ConvJob J = load_job(jr);
  const long C = 1l << logC;
  const int W = 1 << lw;
  const long c0 = col_tile_paired() << lw;
  const Arith<LAZY> A(J.mp);
  u32* __restrict__ c = J.c;
  const int ma = J.ma;
  const int tid = threadIdx.x, nthr = blockDim.x;
  col_dit_rounds<LRB, col_last_round<LRB>(), 0, LAZY>(A, sm, lw, ma << LRB, J.T, tid, nthr, J.Ta, C, c0);
  if constexpr (LRA == 5) {
    // W RB tasks of 32 values on W R / 16 = 2 W RB threads: two lanes per task
    if (ma >= 32 - kFillMax && nthr == 2 * (W << LRB)) {
      const int task = tid >> 1, half = tid & 1;
      const int cc = task & (W - 1);
      const int j1b = task >> lw;
      const uint2* tw = J.T.ri[LRA - 1] + R + j1b * RA + 16 * half;
      u32 x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int ta = 16 * half + i;
        u32 v = 0;
        if (ta < ma) {
          v = sm[((ta * RB + j1b) << lw) + cc];
          if (ta > 0) v = A.mul(v, cld(tw + i));
        }
        x[i] = v;
      }
      switch (ma) {
        case 29: inv32_pair<29, LAZY>(A, x, half, J.T); break;
        case 30: inv32_pair<30, LAZY>(A, x, half, J.T); break;
        case 31: inv32_pair<31, LAZY>(A, x, half, J.T); break;
        default: inv32_pair<32, LAZY>(A, x, half, J.T); break;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = 16 * half + i;
        const long pos = C * (j1b + RB * e) + c0 + cc;
        if (e < ma && pos < J.lc) gst(c + pos, A.canon(TWIST ? A.mul(x[i], cld(J.twi + j1b + RB * e)) : x[i]));
      }
      return;
    }
  }
  for (int task = tid; task < (W << LRB); task += nthr) {
    const int cc = task & (W - 1);
    const int j1b = task >> lw;
    const uint2* tw = J.T.ri[LRA - 1] + R + j1b * RA;
    u32 x[RA];
#pragma unroll
    for (int ta = 0; ta < RA; ++ta) {
      u32 v = 0;
      if (ta < ma) {
        v = sm[((ta * RB + j1b) << lw) + cc];
        if (ta > 0) v = A.mul(v, cld(tw + ta));
      }
      x[ta] = v;
    }
    inv_column<RA, LAZY>(A, x, ma, J.T);
#pragma unroll
    for (int e = 0; e < RA; ++e) {
      const long pos = C * (j1b + RB * e) + c0 + cc;
      if (e < ma && pos < J.lc) gst(c + pos, A.canon(TWIST ? A.mul(x[e], cld(J.twi + j1b + RB * e)) : x[e]));
    }
  }
}

template <int LRA, int LRB, bool TWIST>
static hipError_t col_invr_launch(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  const int lw = col_lw(LRA + LRB, P.logC, (long)njobs);
  const long C = 1l << P.logC;
  if (C < (1l << lw) || col_threads(LRA + LRB, lw) > 1024) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (lw + LRA + LRB)) * sizeof(u32);
  auto kern = k_col_invr<LRA, LRB, kLazy, TWIST>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("col_inv", kern, dim3((unsigned)(C >> lw), 1, njobs), col_threads(LRA + LRB, lw), lds, s, jr,
                P.logC, lw);
}

template <int LRA, bool TWIST>
static hipError_t col_inv_ra(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  const long C = 1l << P.logC;
  if (P.logRB == 0) {
    return launch("col_inv", k_col_inv1<LRA, kLazy, TWIST>, dim3((unsigned)((C + 63) / 64), 1, njobs), 64, 0, s, jr,
                  P.logC);
  }
  if constexpr (LRA >= 4) {
    switch (P.logRB) {
      case 1: return col_invr_launch<LRA, 1, TWIST>(P, jr, njobs, s);
      case 2: return col_invr_launch<LRA, 2, TWIST>(P, jr, njobs, s);
      case 3: return col_invr_launch<LRA, 3, TWIST>(P, jr, njobs, s);
      case 4: return col_invr_launch<LRA, 4, TWIST>(P, jr, njobs, s);
      case 5: return col_invr_launch<LRA, 5, TWIST>(P, jr, njobs, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <bool TWIST>
static hipError_t col_inv_t(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  switch (P.logRA) {
    case 1: return col_inv_ra<1, TWIST>(P, jr, njobs, s);
    case 2: return col_inv_ra<2, TWIST>(P, jr, njobs, s);
    case 3: return col_inv_ra<3, TWIST>(P, jr, njobs, s);
    case 4: return col_inv_ra<4, TWIST>(P, jr, njobs, s);
    case 5: return col_inv_ra<5, TWIST>(P, jr, njobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_col_inv)(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  return P.twist ? col_inv_t<true>(P, jr, njobs, s) : col_inv_t<false>(P, jr, njobs, s);
}

}  // namespace pm
