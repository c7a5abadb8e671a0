// Device building blocks of the transforms: in-register radix-Q DFTs, the
// in-register inverse truncated transform, and the LDS round engine.
//
// Index conventions (section 3 of the paper, eq. 11-14).  A length-N forward
// transform evaluates x(y) = sum_j x_j y^j at the N-th roots of unity.  All
// forward transforms here are decimation-in-frequency networks: natural-order
// input, output slot t holding x(w_N^{rev(t)}) (bit-reversed order).  Cutting
// that output to its first n slots is the truncated Fourier transform
// TFT(N, z, n); the inverse networks take bit-reversed input back to natural
// order.
//
// Twiddle pyramids (one per prime, one per direction) hold Shoup pairs:
//   pf[2^s + x] = (w_{2^s}^x,  floor(w_{2^s}^x * 2^32 / p))      x < 2^s, s <= 15
//   pi[2^s + x] = the same for w_{2^s}^{-x}
//   ph[2^s + x] = w_{2^s}^{-x} / 2                                 s <= 5
//   iv[k]       = 2^-k                                             k <= 32
#pragma once
#include "arith.h"

constexpr int kPyrLog = 15;  // largest pyramid level
constexpr int kPyrSize = 1 << (kPyrLog + 1);
constexpr int kHalfLog = 5;
constexpr int kHalfSize = 1 << (kHalfLog + 1);
constexpr int kInvPow = 33;

// all per-prime constants the kernels read, in one device allocation
struct PrimeTables {
  const uint2* pf;
  const uint2* pi;
  const uint2* ph;
  const uint2* iv;
};

// ---------------------------------------------------------------------------
// In-register transforms of size Q (compile time), values x[0..Q).

// forward DIF: natural in, bit-reversed out
template <int Q, bool LAZY>
__device__ __forceinline__ void dif_reg(const Arith<LAZY>& A, u32* x, const uint2* __restrict__ pf) {
#pragma unroll
  for (int h = Q / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int blk = 0; blk < Q; blk += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        if (i == 0)
          bfly_dif1(A, x[blk + i], x[blk + i + h]);
        else
          bfly_dif(A, x[blk + i], x[blk + i + h], pf[2 * h + i]);
      }
    }
  }
}

// inverse DIT, unscaled (returns Q * x): bit-reversed in, natural out
template <int Q, bool LAZY>
__device__ __forceinline__ void dit_reg(const Arith<LAZY>& A, u32* x, const uint2* __restrict__ pi) {
#pragma unroll
  for (int h = 1; h < Q; h <<= 1) {
#pragma unroll
    for (int blk = 0; blk < Q; blk += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        if (i == 0)
          bfly_dit1(A, x[blk + i], x[blk + i + h]);
        else
          bfly_dit(A, x[blk + i], x[blk + i + h], pi[2 * h + i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// In-register inverse truncated transform (van der Hoeven's ITFT, written as
// a recursion over the DIF network).  Block of N slots starting at OFF.
// On entry: slots i < MK hold the transform outputs (bit-reversed positions),
//           slots i >= MK hold the known inputs (the zero tail at top level).
// On exit:  slots i < MK hold the inputs (the coefficients), scale 1.
// One DIF level maps (a_i, b_i) -> (A_i = a_i + b_i, B_i = (a_i - b_i) w_N^i),
// i < N/2, and then transforms both halves.
//  * MK >= N/2: the left half is fully known at the output, so a full inverse
//    gives A_i; where b_i is known (i >= MK - N/2) this yields a_i and B_i,
//    which are known inputs of the right half; recurse there; then
//    a_i = (A_i + B_i w^-i)/2, b_i = (A_i - B_i w^-i)/2 for the rest.
//  * MK <  N/2: for i >= MK both a_i and b_i are known, so A_i is a known
//    input of the left half; recurse there; then a_i = A_i - b_i.
template <int N, int MK, int OFF, bool LAZY>
struct ItftReg {
  static __device__ __forceinline__ void run(const Arith<LAZY>& A, u32* v, const PrimeTables& T) {
    if constexpr (N == 1 || MK == 0) {
      return;
    } else {
      constexpr int h = N / 2;
      if constexpr (MK >= h) {
        // full scale-1 inverse of the left half
        dit_reg_off<h, OFF>(A, v, T.pi);
        if constexpr (h > 1) {
          const uint2 ih = T.iv[ilog2c(h)];
#pragma unroll
          for (int i = 0; i < h; ++i) v[OFF + i] = A.mul(v[OFF + i], ih);
        }
#pragma unroll
        for (int i = MK - h; i < h; ++i) {
          u32 a = A.sub(v[OFF + i], v[OFF + h + i]);
          u32 d = A.subraw(a, v[OFF + h + i]);
          v[OFF + h + i] = (i == 0) ? A.red(d) : A.mul(d, T.pf[N + i]);
          v[OFF + i] = a;
        }
        ItftReg<h, MK - h, OFF + h, LAZY>::run(A, v, T);
        const uint2 half = T.iv[1];
#pragma unroll
        for (int i = 0; i < MK - h; ++i) {
          u32 t = A.mul(v[OFF + h + i], T.ph[N + i]);
          u32 u = A.mul(v[OFF + i], half);
          v[OFF + i] = A.add(u, t);
          v[OFF + h + i] = A.sub(u, t);
        }
      } else {
#pragma unroll
        for (int i = MK; i < h; ++i) v[OFF + i] = A.add(v[OFF + i], v[OFF + h + i]);
        ItftReg<h, MK, OFF, LAZY>::run(A, v, T);
#pragma unroll
        for (int i = 0; i < MK; ++i) v[OFF + i] = A.sub(v[OFF + i], v[OFF + h + i]);
      }
    }
  }

  template <int Q, int O>
  static __device__ __forceinline__ void dit_reg_off(const Arith<LAZY>& A, u32* v, const uint2* __restrict__ pi) {
#pragma unroll
    for (int hh = 1; hh < Q; hh <<= 1) {
#pragma unroll
      for (int blk = 0; blk < Q; blk += 2 * hh) {
#pragma unroll
        for (int i = 0; i < hh; ++i) {
          if (i == 0)
            bfly_dit1(A, v[O + blk + i], v[O + blk + i + hh]);
          else
            bfly_dit(A, v[O + blk + i], v[O + blk + i + hh], pi[2 * hh + i]);
        }
      }
    }
  }
};

// Dispatch on the runtime number of known outputs m (1 <= m <= Q).  m == Q is
// the full inverse, returned unscaled (Q * x); m < Q returns scale 1.
template <int Q, bool LAZY, int M = 1>
__device__ __forceinline__ void inv_column(const Arith<LAZY>& A, u32* v, int m, const PrimeTables& T) {
  if constexpr (M >= Q) {
    dit_reg<Q>(A, v, T.pi);
  } else {
    if (m == M) {
      ItftReg<Q, M, 0, LAZY>::run(A, v, T);
    } else {
      inv_column<Q, LAZY, M + 1>(A, v, m, T);
    }
  }
}

// ---------------------------------------------------------------------------
// LDS round engine.  The array holds consecutive blocks of size B = 2^LB.
// One round splits every block as index = (B/Q) s + j, s < Q (the top bits):
//   forward: DFT_Q over s (bit-reversed out t), then multiply slot t by
//            w_B^{j rev(t)}; the result in place leaves Q sub-blocks of size B/Q
//            each needing its own length-B/Q transform (section 3, eq. 11).
//   inverse: the mirror image, unscaled.

template <int LB, int LQ, bool LAZY, int NBUF>
__device__ __forceinline__ void dif_round_lds(const Arith<LAZY>& A, u32* const* bufs, int n_el,
                                              const uint2* __restrict__ pf, int tid, int nthr) {
  constexpr int Q = 1 << LQ;
  constexpr int S = 1 << (LB - LQ);
  const int ngroups = n_el >> LQ;
  for (int g = tid; g < ngroups; g += nthr) {
    const int j = g & (S - 1);
    const int base = ((g >> (LB - LQ)) << LB) + j;
    uint2 tw[Q];
    if constexpr (S > 1) {
#pragma unroll
      for (int t = 1; t < Q; ++t) tw[t] = pf[(1 << LB) + j * (int)(__brev((u32)t) >> (32 - LQ))];
    }
#pragma unroll
    for (int bi = 0; bi < NBUF; ++bi) {
      u32* buf = bufs[bi];
      u32 x[Q];
#pragma unroll
      for (int s = 0; s < Q; ++s) x[s] = buf[base + S * s];
      dif_reg<Q>(A, x, pf);
      if constexpr (S > 1) {
#pragma unroll
        for (int t = 1; t < Q; ++t) x[t] = A.mul(x[t], tw[t]);
      }
#pragma unroll
      for (int t = 0; t < Q; ++t) buf[base + S * t] = x[t];
    }
  }
}

template <int LB, int LQ, bool LAZY>
__device__ __forceinline__ void dit_round_lds(const Arith<LAZY>& A, u32* buf, int n_el, const uint2* __restrict__ pi,
                                              int tid, int nthr) {
  constexpr int Q = 1 << LQ;
  constexpr int S = 1 << (LB - LQ);
  const int ngroups = n_el >> LQ;
  for (int g = tid; g < ngroups; g += nthr) {
    const int j = g & (S - 1);
    const int base = ((g >> (LB - LQ)) << LB) + j;
    u32 x[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) x[t] = buf[base + S * t];
    if constexpr (S > 1) {
#pragma unroll
      for (int t = 1; t < Q; ++t) x[t] = A.mul(x[t], pi[(1 << LB) + j * (int)(__brev((u32)t) >> (32 - LQ))]);
    }
    dit_reg<Q>(A, x, pi);
#pragma unroll
    for (int s = 0; s < Q; ++s) buf[base + S * s] = x[s];
  }
}

// forward transform of every block of size 2^LB in the buffers (n_el elements
// each); ends with a barrier
template <int LB, int LQMAX, bool LAZY, int NBUF>
__device__ __forceinline__ void dif_lds(const Arith<LAZY>& A, u32* const* bufs, int n_el, const uint2* __restrict__ pf,
                                        int tid, int nthr) {
  if constexpr (LB > 0) {
    constexpr int LQ = LB < LQMAX ? LB : LQMAX;
    dif_round_lds<LB, LQ, LAZY, NBUF>(A, bufs, n_el, pf, tid, nthr);
    __syncthreads();
    dif_lds<LB - LQ, LQMAX, LAZY, NBUF>(A, bufs, n_el, pf, tid, nthr);
  }
}

// inverse (unscaled) of dif_lds; ends with a barrier
template <int LB, int LQMAX, bool LAZY>
__device__ __forceinline__ void dit_lds(const Arith<LAZY>& A, u32* buf, int n_el, const uint2* __restrict__ pi, int tid,
                                        int nthr) {
  if constexpr (LB > 0) {
    constexpr int LQ = LB < LQMAX ? LB : LQMAX;
    dit_lds<LB - LQ, LQMAX, LAZY>(A, buf, n_el, pi, tid, nthr);
    dit_round_lds<LB, LQ, LAZY>(A, buf, n_el, pi, tid, nthr);
    __syncthreads();
  }
}
