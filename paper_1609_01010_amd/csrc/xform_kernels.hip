// Standalone transforms behind the test hooks pm_ntt, pm_tft and pm_itft:
// the modular DFT in natural order (section 3), the truncated transform TFT
// in bit-reversed order and its inverse ITFT scaled by L (the TFT product,
// eq. 14).  They reuse the convolution's building blocks.
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
// one work-group, L = 2^LN <= 2^14, first radix RA (truncated to ma blocks)

template <int LN, int LRA, bool LAZY>
__global__ void __launch_bounds__(1024) k_lds_xform(const u32* in, int zin, u32* out, int nout,
                                                    int ma, int dir, int natural, ModP mp, PrimeTables T, uint2 sc,
                                                    int* err) {
  constexpr int N = 1 << LN;
  constexpr int RA = 1 << LRA;
  constexpr int LS = LN - LRA;
  constexpr int S = 1 << LS;
  extern __shared__ u32 sm[];
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nel = ma * S;
  bool bad = false;
  if (dir == 0) {
    for (int j = tid; j < S; j += nthr) {
      u32 x[RA];
#pragma unroll
      for (int s = 0; s < RA; ++s) {
        const int pos = j + S * s;
        x[s] = pos < zin ? in[pos] : 0u;
        bad |= x[s] >= mp.p;
      }
      dif_reg<RA>(A, x, T.pf);
#pragma unroll
      for (int t = 0; t < RA; ++t) {
        if (t < ma) {
          u32 v = x[t];
          if constexpr (S > 1) {
            if (t > 0) v = A.mul(v, cld(T.rf[LRA - 1] + N + j * RA + t));
          }
          sm[lds_ix(j + S * t)] = v;
        }
      }
    }
    __syncthreads();
    u32* bufs[1] = {sm};
    dif_lds<LS, 4, LAZY, 1>(A, bufs, nel, T, tid, nthr);
    if (natural) {
      for (int k = tid; k < N; k += nthr) out[k] = A.canon(sm[lds_ix(bitrev_n((u32)k, LN))]);
    } else {
      for (int i = tid; i < nout; i += nthr) out[i] = A.canon(sm[lds_ix(i)]);
    }
  } else {
    if (natural) {
      for (int t = tid; t < N; t += nthr) {
        const u32 v = in[bitrev_n((u32)t, LN)];
        bad |= v >= mp.p;
        sm[lds_ix(t)] = v;
      }
    } else {
      for (int i = tid; i < nel; i += nthr) {
        const u32 v = in[i];
        bad |= v >= mp.p;
        sm[lds_ix(i)] = v;
      }
    }
    __syncthreads();
    dit_lds<LS, 4, LAZY>(A, sm, nel, T, tid, nthr);
    for (int j = tid; j < S; j += nthr) {
      u32 x[RA];
#pragma unroll
      for (int t = 0; t < RA; ++t) {
        u32 v = 0;
        if (t < ma) {
          v = sm[lds_ix(j + S * t)];
          if constexpr (S > 1) {
            if (t > 0) v = A.mul(v, cld(T.ri[LRA - 1] + N + j * RA + t));
          }
        }
        x[t] = v;
      }
      inv_column<RA, LAZY>(A, x, ma, T);
#pragma unroll
      for (int s = 0; s < RA; ++s) {
        const int pos = j + S * s;
        if (s < ma && pos < nout) out[pos] = A.canon(A.mul(x[s], sc));
      }
    }
  }
  if (bad) atomicOr(err, 1);
}

template <int LN, int LRA, bool LAZY>
static hipError_t lds_xform_inst(const Plan& P, const u32* in, long zin, u32* out, long nout, int dir, int natural,
                                 const ModP& mp, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  constexpr int N = 1 << LN;
  int nthr = N / 16;
  if (nthr < 64) nthr = 64;
  if (nthr > 1024) nthr = 1024;
  const size_t lds = (size_t)N * sizeof(u32);
  auto kern = k_lds_xform<LN, LRA, LAZY>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("lds_xform", kern, 1, nthr, lds, s, in, (int)zin, out, (int)nout, P.ma, dir, natural, mp, T, sc, err);
}

template <int LN, bool LAZY>
static hipError_t lds_xform_ln(const Plan& P, const u32* in, long zin, u32* out, long nout, int dir, int natural,
                               const ModP& mp, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  // the hooks use the first radix min(32, L)
  constexpr int LRA = LN < 5 ? LN : 5;
  if (P.logRA != LRA) return hipErrorInvalidValue;
  return lds_xform_inst<LN, LRA, LAZY>(P, in, zin, out, nout, dir, natural, mp, T, sc, err, s);
}

hipError_t PM_SUFFIX(launch_lds_xform)(const Plan& P, const u32* in, long zin, u32* out, long nout, int dir, int natural,
                            int pidx, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  const ModP mp = modp_of(PI);
#define PM_LN(n)                                                                                   \
  case n:                                                                                          \
    return lds_xform_ln<n, kLazy>(P, in, zin, out, nout, dir, natural, mp, T, sc, err, s);
  switch (P.logL) {
    PM_LN(1) PM_LN(2) PM_LN(3) PM_LN(4) PM_LN(5) PM_LN(6) PM_LN(7) PM_LN(8) PM_LN(9) PM_LN(10) PM_LN(11)
    PM_LN(12) PM_LN(13) PM_LN(14)
    default:
      break;
  }
#undef PM_LN
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// four-step row transforms (one operand): forward = twiddle by w_L^{j2 k1}
// then DIF; inverse = DIT, then untwiddle by w_L^{-j2 k1} times the scale
// folded into the row tables.  As in the convolution's row pass, the
// outermost round runs in registers beside the coalesced load (forward) or
// store (inverse) and the innermost one beside the contiguous store (forward)
// or load (inverse); the rounds between use LDS.

template <int LC, int LNT, int LQ, bool LAZY>
__global__ void __launch_bounds__(1 << LNT) k_row_fwd(const u32* in, u32* out, long nout, int logR, ModP mp,
                                                      PrimeTables T, RowTables W) {
  constexpr int C = 1 << LC;
  constexpr int NT = 1 << LNT;
  constexpr int LE = LC - LNT;
  constexpr int EPT = 1 << LE;
  constexpr int LQL = last_lb<LNT, LQ>();
  constexpr int QL = 1 << LQL;
  extern __shared__ u32 sm[];
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x;
  const int row = blockIdx.x;
  const u32 k1 = bitrev_n((u32)row, logR);
  const long off = (long)row * C;
  const uint2 gf = cld(W.gf + k1 * (u32)NT + tid);
  const uint2* ff = W.ff + (size_t)k1 * EPT;
  u32 x[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) x[e] = in[off + tid + NT * e];
  row_twist_fwd<LC, LE, LAZY>(A, x, gf, ff, T, tid);
#pragma unroll
  for (int t = 0; t < EPT; ++t) sm[lds_ix(tid + NT * t)] = x[t];
  __syncthreads();
  u32* bufs[1] = {sm};
  dif_lds_upto<LNT, LQL, LQ, LAZY, 1>(A, bufs, C, T, tid, NT);
#pragma unroll
  for (int u = 0; u < EPT / QL; ++u) {
    const long base = off + (long)(tid + NT * u) * QL;
    u32 y[QL];
    lds_load_contig<QL>(sm, (tid + NT * u) * QL, y);
    dif_reg<QL>(A, y, T.pf);
    if (base + QL <= nout) {
#pragma unroll
      for (int t = 0; t < QL; ++t) out[base + t] = A.canon(y[t]);
    } else {
#pragma unroll
      for (int t = 0; t < QL; ++t)
        if (base + t < nout) out[base + t] = A.canon(y[t]);
    }
  }
}

template <int LC, int LNT, int LQ, bool LAZY>
__global__ void __launch_bounds__(1 << LNT) k_row_inv(const u32* in, u32* out, int logR, ModP mp, PrimeTables T,
                                                      RowTables W) {
  constexpr int C = 1 << LC;
  constexpr int NT = 1 << LNT;
  constexpr int LE = LC - LNT;
  constexpr int EPT = 1 << LE;
  constexpr int LQL = last_lb<LNT, LQ>();
  constexpr int QL = 1 << LQL;
  extern __shared__ u32 sm[];
  const Arith<LAZY> A(mp);
  const int tid = threadIdx.x;
  const int row = blockIdx.x;
  const u32 k1 = bitrev_n((u32)row, logR);
  const long off = (long)row * C;
#pragma unroll
  for (int u = 0; u < EPT / QL; ++u) {
    const long base = off + (long)(tid + NT * u) * QL;
    u32 y[QL];
#pragma unroll
    for (int t = 0; t < QL; ++t) y[t] = in[base + t];
    dit_reg<QL>(A, y, T.pi);
    lds_store_contig<QL>(sm, (tid + NT * u) * QL, y);
  }
  __syncthreads();
  dit_lds_from<LNT, LQL, LQ, LAZY>(A, sm, C, T, tid, NT);
  u32 x[EPT];
#pragma unroll
  for (int t = 0; t < EPT; ++t) x[t] = sm[lds_ix(tid + NT * t)];
  dit_top_reg<LC, LE, LAZY>(A, x, T, tid);
  const uint2 gi = cld(W.gi + k1 * (u32)NT + tid);
  const uint2* fi = W.fi + (size_t)k1 * EPT;
#pragma unroll
  for (int e = 0; e < EPT; ++e) out[off + tid + NT * e] = A.mul(A.mul_raw(x[e], gi), cld(fi + e));
}

template <int LC, bool LAZY>
static hipError_t row_xform_inst(const Plan& P, const u32* in, u32* out, long nout, int dir, const ModP& mp,
                                 const PrimeTables& T, const RowTables& W, hipStream_t s) {
  constexpr int C = 1 << LC;
  constexpr int LNT = LC - 4;
  if (plan_row_lnt(P) != LNT) return hipErrorInvalidValue;
  const int rows = P.ma << P.logRB;
  const int logR = P.logRA + P.logRB;
  const size_t lds = (size_t)C * sizeof(u32);
  if (dir == 0) {
    auto kern = k_row_fwd<LC, LNT, 3, LAZY>;
    ensure_lds_attr((const void*)kern, lds);
    return launch("row_xform", kern, rows, 1 << LNT, lds, s, in, out, nout, logR, mp, T, W);
  }
  auto kern = k_row_inv<LC, LNT, 3, LAZY>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("row_xform", kern, rows, 1 << LNT, lds, s, in, out, logR, mp, T, W);
}

hipError_t PM_SUFFIX(launch_row_xform)(const Plan& P, const u32* in, u32* out, long nout, int dir, int pidx,
                                       const PrimeTables& T, const RowTables& W, hipStream_t s) {
  const ModP mp = modp_of(prime_info(pidx));
  switch (P.logC) {
#define PM_LC(n) \
  case n:        \
    return row_xform_inst<n, kLazy>(P, in, out, nout, dir, mp, T, W, s);
    PM_LC(10) PM_LC(11) PM_LC(12) PM_LC(13) PM_LC(14)
#undef PM_LC
    default:
      break;
  }
  return hipErrorInvalidValue;
}

#if PM_LAZY == 1
// ---------------------------------------------------------------------------
// layout changes for the natural-order hooks: the four-step layout holds
// X_{k1 + R k2} at row t1 = rev_r(k1), column t2 = rev_c(k2).

__global__ void k_permute(const u32* __restrict__ in, u32* __restrict__ out, int logR, int logC, int to_natural) {
  const long n = 1l << (logR + logC);
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // i: flat index in the four-step layout
  const u32 t1 = (u32)(i >> logC), t2 = (u32)(i & ((1l << logC) - 1));
  const long k = (long)bitrev_n(t1, logR) + ((long)bitrev_n(t2, logC) << logR);
  if (to_natural)
    out[k] = in[i];
  else
    out[i] = in[k];
}

hipError_t launch_permute(const u32* in, u32* out, int logR, int logC, int to_natural, hipStream_t s) {
  const long n = 1l << (logR + logC);
  return launch("permute", k_permute, (unsigned)((n + 255) / 256), 256, 0, s, in, out, logR, logC, to_natural);
}

#endif

}  // namespace pm
