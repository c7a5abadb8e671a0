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
// one work-group per product, everything in LDS (L = 2^LN <= 2^14).
// The first round (radix RA over the top log2 RA index bits) is done in
// registers straight from global memory and keeps the first ma of its RA
// output blocks; the remaining rounds transform those blocks in LDS.

template <int LN, int LRA, int LQ, bool LAZY, bool TWIST>
__device__ __forceinline__ void lds_conv_body(const ConvJob& J, u32* sm) {
  constexpr int N = 1 << LN;
  constexpr int RA = 1 << LRA;
  constexpr int LS = LN - LRA;
  constexpr int S = 1 << LS;
  const u32* __restrict__ a = (const u32*)J.a;
  const u32* __restrict__ b = (const u32*)J.b;
  const int la = (int)J.la, lb = (int)J.lb, lc = (int)J.lc, ma = J.ma;
  const PrimeTables& T = J.T;
  u32* sa = sm;
  u32* sb = sm + N;
  const Arith<LAZY> A(J.mp);
  const int tid = threadIdx.x, nthr = blockDim.x;
  bool bad = false;

  // The columns of both operands: side by side when there are threads for
  // all 2S of them (a product on its own, bound by latency), else one
  // operand after the other (the twiddles of a column are then read again,
  // from cache, rather than held in registers across both).
  const bool side = nthr >= 2 * S;
  for (int pass = 0; pass < (side ? 1 : 2); ++pass) {
    for (int w = tid; w < (side ? 2 * S : S); w += nthr) {
      const int op = side ? w / S : pass;
      const int j = side ? w % S : w;
      const u32* in = op ? b : a;
      const int len = op ? lb : la;
      u32* out = op ? sb : sa;
      const uint2* tw = T.rf[LRA - 1] + N + j * RA;
      u32 x[RA];
#pragma unroll
      for (int s = 0; s < RA; ++s) {
        const int pos = j + S * s;
        x[s] = pos < len ? gld(in + pos) : 0u;
        bad |= x[s] >= J.mp.p;
        if constexpr (TWIST) x[s] = A.mul(x[s], cld(J.twf + pos));
      }
      dif_reg<RA, LAZY, (S > 1)>(A, x, T.pf);
#pragma unroll
      for (int t = 0; t < RA; ++t) {
        if (t < ma) {
          u32 v = x[t];
          if constexpr (S > 1) {
            if (t > 0) v = A.mul(v, cld(tw + t));
          }
          out[lds_ix(j + S * t)] = v;
        }
      }
    }
  }
  if (bad) atomicOr(J.err, 1);
  __syncthreads();
  const int nel = ma * S;
  constexpr int LQL = last_lb<LS, LQ>();
  u32* bufs[2] = {sa, sb};
  dif_lds_upto<LS, LQL, LQ, LAZY, 2>(A, bufs, nel, T, tid, nthr);
  conv_inner<LQL, LAZY>(A, sa, sb, nel, T, tid, nthr, J.sc);
  __syncthreads();
  dit_lds_from<LS, LQL, LQ, LAZY>(A, sa, nel, T, tid, nthr);
  u32* __restrict__ c = J.c;
  for (int j = tid; j < S; j += nthr) {
    const uint2* tw = T.ri[LRA - 1] + N + j * RA;
    u32 x[RA];
#pragma unroll
    for (int t = 0; t < RA; ++t) {
      u32 v = 0;
      if (t < ma) {
        v = sa[lds_ix(j + S * t)];
        if constexpr (S > 1) {
          if (t > 0) v = A.mul(v, cld(tw + t));
        }
      }
      x[t] = v;
    }
    inv_column<RA, LAZY>(A, x, ma, T);
#pragma unroll
    for (int s = 0; s < RA; ++s) {
      const int pos = j + S * s;
      if (s < ma && pos < lc) gst(c + pos, A.canon(TWIST ? A.mul(x[s], cld(J.twi + pos)) : x[s]));
    }
  }
}

template <int LN, int LRA, int LQ, bool LAZY, bool TWIST>
__global__ void __launch_bounds__(1024) k_lds_conv(JobRef jr) {
  extern __shared__ u32 sm[];
  const ConvJob J = load_job(jr);
  lds_conv_body<LN, LRA, LQ, LAZY, TWIST>(J, sm);
}

// The same for a batch's products of several lengths up to 2^kMultiMaxLN,
// first radix 8 (the default and the tuner's usual pick there), in one
// launch: work-group z takes job z and runs the body of its own length (from
// the descriptor); the work-group has the threads and LDS of the longest.
// (The bodies of the larger first radices carry the truncated inverse for
// every count of kept blocks, whose registers would spill here.)
constexpr int kMultiMaxLN = 11;
constexpr int kMultiThreads = 128;

template <bool LAZY>
__global__ void __launch_bounds__(kMultiThreads) k_lds_conv_multi(JobRef jr) {
  extern __shared__ u32 sm[];
  const ConvJob J = load_job(jr);
  switch (J.logL) {
#define PM_BODY(ln)                                     \
  case ln:                                              \
    lds_conv_body<ln, 3, 4, LAZY, false>(J, sm);        \
    break;
    PM_BODY(6) PM_BODY(7) PM_BODY(8) PM_BODY(9) PM_BODY(10) PM_BODY(11)
#undef PM_BODY
    default:
      break;
  }
}

// whether a one-work-group plan may run in the several-length launch
bool PM_SUFFIX(lds_multi_ok)(const Plan& P) {
  return P.kind == PLAN_LDS && !P.twist && P.logL >= 6 && P.logL <= kMultiMaxLN && P.logRA == 3;
}

hipError_t PM_SUFFIX(launch_lds_conv_multi)(const JobRef& jr, int njobs, hipStream_t s) {
  const size_t lds = 2 * ((size_t)1 << kMultiMaxLN) * sizeof(u32);
  auto kern = k_lds_conv_multi<kLazy>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("lds_conv", kern, dim3(1, 1, njobs), kMultiThreads, lds, s, jr);
}

// threads of the one-work-group convolution of length 2^ln: 16 values per
// thread in a batch (several work-groups share a compute unit), 4 for a
// product on its own, which has the compute unit to itself and is bound by
// the latency of its rounds
inline int lds_conv_threads(int ln, int njobs) {
  int nthr = (1 << ln) / (njobs == 1 ? 4 : 16);
  return nthr < 64 ? 64 : (nthr > 1024 ? 1024 : nthr);
}

template <int LN, int LRA, bool TWIST>
static hipError_t lds_conv_inst(const JobRef& jr, int njobs, hipStream_t s) {
  constexpr int N = 1 << LN;
  const size_t lds = 2 * (size_t)N * sizeof(u32);
  auto kern = k_lds_conv<LN, LRA, 4, kLazy, TWIST>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("lds_conv", kern, dim3(1, 1, njobs), lds_conv_threads(LN, njobs), lds, s, jr);
}

// the nega-circular products (twisted) use the first radix 16 only
template <int LN>
static hipError_t lds_conv_ra(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
  if (P.twist) return P.logRA == 4 ? lds_conv_inst<LN, 4, true>(jr, njobs, s) : hipErrorInvalidValue;
  switch (P.logRA) {
#define PM_RA(r)                                                                    \
  case r:                                                                           \
    if constexpr (r <= LN) return lds_conv_inst<LN, r, false>(jr, njobs, s);        \
    break;
    PM_RA(3) PM_RA(4) PM_RA(5)
#undef PM_RA
    default:
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t PM_SUFFIX(launch_lds_conv)(const Plan& P, const JobRef& jr, int njobs, hipStream_t s) {
#define PM_LN(n) \
  case n:        \
    return lds_conv_ra<n>(P, jr, njobs, s);
  switch (P.logL) {
    PM_LN(6) PM_LN(7) PM_LN(8) PM_LN(9) PM_LN(10) PM_LN(11) PM_LN(12) PM_LN(13) PM_LN(14)
    default:
      break;
  }
#undef PM_LN
  return hipErrorInvalidValue;
}

}  // namespace pm
