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
// Round tables, for radix Q = 2^q (q = 1 .. 6), level B = 2^s >= Q:
//   rf[q-1][B + j Q + t] = w_B^{j rev_q(t)},  j < B/Q, t < Q   (ri: w_B^{-j rev_q(t)})
// so the Q twiddles of one group of an LDS round are 8Q contiguous bytes.
#pragma once
#include "arith.h"

constexpr int kPyrLog = 15;  // largest pyramid level
constexpr int kPyrSize = 1 << (kPyrLog + 1);
constexpr int kHalfLog = 5;
constexpr int kHalfSize = 1 << (kHalfLog + 1);
constexpr int kInvPow = 33;
constexpr int kRoundTables = 6;  // radices 2 .. 64

// Completion matrices of truncated inverses (itft_fill): for Q = 2^q,
// q = kFillMinLog .. kFillMaxLog, and d = 1 .. kFillMax unknown outputs, the
// d x (Q - d) matrix K, row-major, with x[Q - d + r] = sum_k K[r][k] x[k].
constexpr int kFillMax = 3;
constexpr int kFillMinLog = 3;
constexpr int kFillMaxLog = 5;
__host__ __device__ constexpr int fill_offset(int lq, int d) {
  int off = 0;
  for (int q = kFillMinLog; q <= kFillMaxLog + 1; ++q)
    for (int e = 1; e <= kFillMax; ++e) {
      if (q == lq && e == d) return off;
      off += e * ((1 << q) - e);
    }
  return off;
}
constexpr int kFillSize = fill_offset(kFillMaxLog + 1, 1);

// all per-prime constants the kernels read, in one device allocation
struct PrimeTables {
  const uint2* pf;
  const uint2* pi;
  const uint2* ph;
  const uint2* iv;
  const uint2* rf[kRoundTables];
  const uint2* ri[kRoundTables];
  const uint2* kx;  // completion matrices (kFillSize pairs)
};

// the same tables, reads not merged with those before this point (see fresh)
__device__ __forceinline__ PrimeTables fresh(const PrimeTables& T) {
  PrimeTables R;
  R.pf = fresh(T.pf);
  R.pi = fresh(T.pi);
  R.ph = fresh(T.ph);
  R.iv = fresh(T.iv);
  R.kx = fresh(T.kx);
#pragma unroll
  for (int q = 0; q < kRoundTables; ++q) {
    R.rf[q] = fresh(T.rf[q]);
    R.ri[q] = fresh(T.ri[q]);
  }
  return R;
}

// ---------------------------------------------------------------------------
// In-register transforms of size Q (compile time), values x[0..Q).

// forward DIF: natural in, bit-reversed out.  RAW_TAIL: outputs 1..Q-1 are
// left in [0, 2K) (for a caller that multiplies each of them next); output 0
// is always reduced.  HZ: the caller guarantees x[Q/2..Q) = 0 (an operand
// shorter than half the transform), so the first level is (a, 0) -> (a, a w)
// with no sum or difference.
template <int Q, bool LAZY, bool RAW_TAIL = false, bool HZ = false>
__device__ __forceinline__ void dif_reg(const Arith<LAZY>& A, u32* x, const uint2* __restrict__ pf) {
#pragma unroll
  for (int h = Q / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int blk = 0; blk < Q; blk += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        if (HZ && h == Q / 2)
          x[i + h] = i == 0 ? x[i] : A.mul(x[i], cld(pf + 2 * h + i));
        else if (i != 0)
          bfly_dif(A, x[blk + i], x[blk + i + h], cld(pf + 2 * h + i));
        else if (RAW_TAIL && h == 1 && blk > 0)
          bfly_dif1_raw(A, x[blk], x[blk + 1]);
        else if (RAW_TAIL && h == 1) {
          const u32 a = x[0], b = x[1];
          x[0] = A.add(a, b);
          x[1] = A.subraw(a, b);
        } else
          bfly_dif1(A, x[blk + i], x[blk + i + h]);
      }
    }
  }
}

// inverse DIT, unscaled (returns Q * x): bit-reversed in, natural out.
// RAW_OUT: all outputs left in [0, 2K) (for a caller that multiplies each of
// them next).
template <int Q, bool LAZY, bool RAW_OUT = false>
__device__ __forceinline__ void dit_reg(const Arith<LAZY>& A, u32* x, const uint2* __restrict__ pi) {
#pragma unroll
  for (int h = 1; h < Q; h <<= 1) {
#pragma unroll
    for (int blk = 0; blk < Q; blk += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        if (RAW_OUT && 2 * h == Q) {
          if (i == 0)
            bfly_dit1_raw(A, x[blk + i], x[blk + i + h]);
          else
            bfly_dit_raw(A, x[blk + i], x[blk + i + h], cld(pi + 2 * h + i));
        } else if (i == 0)
          bfly_dit1(A, x[blk + i], x[blk + i + h]);
        else
          bfly_dit(A, x[blk + i], x[blk + i + h], cld(pi + 2 * h + i));
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
          const uint2 ih = cld(T.iv + ilog2c(h));
#pragma unroll
          for (int i = 0; i < h; ++i) v[OFF + i] = A.mul(v[OFF + i], ih);
        }
#pragma unroll
        for (int i = MK - h; i < h; ++i) {
          u32 a = A.sub(v[OFF + i], v[OFF + h + i]);
          u32 d = A.subraw(a, v[OFF + h + i]);
          v[OFF + h + i] = (i == 0) ? A.red(d) : A.mul(d, cld(T.pf + N + i));
          v[OFF + i] = a;
        }
        ItftReg<h, MK - h, OFF + h, LAZY>::run(A, v, T);
        const uint2 half = cld(T.iv + 1);
#pragma unroll
        for (int i = 0; i < MK - h; ++i) {
          u32 t = A.mul(v[OFF + h + i], cld(T.ph + N + i));
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
            bfly_dit(A, v[O + blk + i], v[O + blk + i + hh], cld(pi + 2 * hh + i));
        }
      }
    }
  }
};

// The same inverse when only d = Q - M outputs are unknown (d small): the
// coefficients at j >= M are zero, and these d equations fix the unknown
// outputs as linear combinations of the known ones, x[M + r] = sum_k K[r][k]
// x[k] (K = -G_m^-1 G_k from the inverse transform matrix G, computed on the
// host).  Then one full inverse network and the factor Q^-1.  Same contract
// as ItftReg; more arithmetic than the recursion, but every step has the full
// network's independent butterflies instead of a chain of shrinking
// transforms, which is what limits a thread that runs the recursion alone.
template <int Q, int M, bool LAZY>
__device__ __forceinline__ void itft_fill(const Arith<LAZY>& A, u32* v, const PrimeTables& T) {
  constexpr int D = Q - M;
  const uint2* K = T.kx + fill_offset(ilog2c(Q), D);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    u32 acc = A.mul(v[0], cld(K + r * M));
#pragma unroll
    for (int k = 1; k < M; ++k) acc = A.add(acc, A.mul(v[k], cld(K + r * M + k)));
    v[M + r] = acc;
  }
  dit_reg<Q>(A, v, T.pi);
  const uint2 qi = cld(T.iv + ilog2c(Q));
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = A.mul(v[j], qi);
}

// Dispatch on the runtime number of known outputs m (1 <= m <= Q).  m == Q is
// the full inverse, returned unscaled (Q * x); m < Q returns scale 1.
template <int Q, bool LAZY, int M = 1>
__device__ __forceinline__ void inv_column(const Arith<LAZY>& A, u32* v, int m, const PrimeTables& T) {
  if constexpr (M >= Q) {
    dit_reg<Q>(A, v, T.pi);
  } else {
    if (m == M) {
      if constexpr (Q >= (1 << kFillMinLog) && Q <= (1 << kFillMaxLog) && Q - M <= kFillMax)
        itft_fill<Q, M, LAZY>(A, v, T);
      else
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
// LDS addresses are swizzled (bits 2-4 ^= bits 6-8): the rounds whose groups
// are 64 words apart would otherwise hit one bank of the 32; aligned quads
// stay aligned, so the contiguous groups of the last round load as 16 bytes.

__device__ __forceinline__ int lds_ix(int a) { return a ^ (((a >> 6) & 7) << 2); }

template <int Q>
__device__ __forceinline__ void load_tw(uint2 (&tw)[Q], const uint2* __restrict__ p) {
  const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int t = 0; t < Q / 2; ++t) {
    const uint4 v = cld(q + t);
    tw[2 * t] = make_uint2(v.x, v.y);
    tw[2 * t + 1] = make_uint2(v.z, v.w);
  }
}

// Q contiguous words at position `base` (multiple of Q)
template <int Q>
__device__ __forceinline__ void lds_load_contig(const u32* buf, int base, u32 (&x)[Q]) {
  if constexpr (Q >= 4) {
#pragma unroll
    for (int k = 0; k < Q; k += 4) {
      const uint4 v = *reinterpret_cast<const uint4*>(buf + lds_ix(base + k));
      x[k] = v.x;
      x[k + 1] = v.y;
      x[k + 2] = v.z;
      x[k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) x[k] = buf[lds_ix(base + k)];
  }
}
template <int Q>
__device__ __forceinline__ void lds_store_contig(u32* buf, int base, const u32 (&x)[Q]) {
  if constexpr (Q >= 4) {
#pragma unroll
    for (int k = 0; k < Q; k += 4)
      *reinterpret_cast<uint4*>(buf + lds_ix(base + k)) = make_uint4(x[k], x[k + 1], x[k + 2], x[k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) buf[lds_ix(base + k)] = x[k];
  }
}

template <int LB, int LQ, bool LAZY, int NBUF>
__device__ __forceinline__ void dif_round_lds(const Arith<LAZY>& A, u32* const* bufs, int n_el,
                                              const PrimeTables& T, int tid, int nthr) {
  constexpr int Q = 1 << LQ;
  constexpr int S = 1 << (LB - LQ);
  const int ngroups = n_el >> LQ;
  for (int g = tid; g < ngroups; g += nthr) {
    const int j = g & (S - 1);
    const int base = ((g >> (LB - LQ)) << LB) + j;
    uint2 tw[Q];
    if constexpr (S > 1) load_tw<Q>(tw, T.rf[LQ - 1] + (1 << LB) + j * Q);
#pragma unroll
    for (int bi = 0; bi < NBUF; ++bi) {
      u32* buf = bufs[bi];
      u32 x[Q];
      if constexpr (S == 1) {
        lds_load_contig<Q>(buf, base, x);
      } else {
#pragma unroll
        for (int s = 0; s < Q; ++s) x[s] = buf[lds_ix(base + S * s)];
      }
      dif_reg<Q, LAZY, (S > 1)>(A, x, T.pf);
      if constexpr (S > 1) {
#pragma unroll
        for (int t = 1; t < Q; ++t) x[t] = A.mul(x[t], tw[t]);
#pragma unroll
        for (int t = 0; t < Q; ++t) buf[lds_ix(base + S * t)] = x[t];
      } else {
        lds_store_contig<Q>(buf, base, x);
      }
    }
  }
}

template <int LB, int LQ, bool LAZY>
__device__ __forceinline__ void dit_round_lds(const Arith<LAZY>& A, u32* buf, int n_el, const PrimeTables& T, int tid,
                                              int nthr) {
  constexpr int Q = 1 << LQ;
  constexpr int S = 1 << (LB - LQ);
  const int ngroups = n_el >> LQ;
  for (int g = tid; g < ngroups; g += nthr) {
    const int j = g & (S - 1);
    const int base = ((g >> (LB - LQ)) << LB) + j;
    u32 x[Q];
    if constexpr (S == 1) {
      lds_load_contig<Q>(buf, base, x);
    } else {
      uint2 tw[Q];
      load_tw<Q>(tw, T.ri[LQ - 1] + (1 << LB) + j * Q);
#pragma unroll
      for (int t = 0; t < Q; ++t) x[t] = buf[lds_ix(base + S * t)];
#pragma unroll
      for (int t = 1; t < Q; ++t) x[t] = A.mul(x[t], tw[t]);
    }
    dit_reg<Q>(A, x, T.pi);
    if constexpr (S == 1) {
      lds_store_contig<Q>(buf, base, x);
    } else {
#pragma unroll
      for (int s = 0; s < Q; ++s) buf[lds_ix(base + S * s)] = x[s];
    }
  }
}

// radix of the round that starts at block size 2^LB: the remainder of LB
// modulo LQMAX first, then rounds of radix 2^LQMAX, so that the innermost
// round (contiguous groups) is a full one
template <int LB, int LQMAX>
constexpr int round_lq() {
  return LB % LQMAX == 0 ? LQMAX : LB % LQMAX;
}

// forward transform of every block of size 2^LB in the buffers (n_el
// elements each); ends with a barrier.  Rounds of radix 2^LQMAX, the last
// one smaller if LB is not a multiple of LQMAX.
template <int LB, int LQMAX, bool LAZY, int NBUF>
__device__ __forceinline__ void dif_lds(const Arith<LAZY>& A, u32* const* bufs, int n_el, const PrimeTables& T,
                                        int tid, int nthr) {
  if constexpr (LB > 0) {
    constexpr int LQ = round_lq<LB, LQMAX>();
    dif_round_lds<LB, LQ, LAZY, NBUF>(A, bufs, n_el, T, tid, nthr);
    __syncthreads();
    dif_lds<LB - LQ, LQMAX, LAZY, NBUF>(A, bufs, n_el, T, tid, nthr);
  }
}

// inverse (unscaled) of dif_lds; ends with a barrier
template <int LB, int LQMAX, bool LAZY>
__device__ __forceinline__ void dit_lds(const Arith<LAZY>& A, u32* buf, int n_el, const PrimeTables& T, int tid,
                                        int nthr) {
  if constexpr (LB > 0) {
    constexpr int LQ = round_lq<LB, LQMAX>();
    dit_lds<LB - LQ, LQMAX, LAZY>(A, buf, n_el, T, tid, nthr);
    dit_round_lds<LB, LQ, LAZY>(A, buf, n_el, T, tid, nthr);
    __syncthreads();
  }
}

// forward rounds on blocks of size 2^LB down to block size 2^LSTOP, in each
// of NBUF buffers; ends with a barrier (none if there is no round)
template <int LB, int LSTOP, int LQMAX, bool LAZY, int NBUF = 1>
__device__ __forceinline__ void dif_lds_upto(const Arith<LAZY>& A, u32* const* bufs, int n_el, const PrimeTables& T,
                                             int tid, int nthr) {
  if constexpr (LB > LSTOP) {
    constexpr int LQ = round_lq<LB, LQMAX>();
    dif_round_lds<LB, LQ, LAZY, NBUF>(A, bufs, n_el, T, tid, nthr);
    __syncthreads();
    dif_lds_upto<LB - LQ, LSTOP, LQMAX, LAZY, NBUF>(A, bufs, n_el, T, tid, nthr);
  }
}

// inverse rounds for block sizes above 2^LSTOP up to 2^LB; ends with a barrier
template <int LB, int LSTOP, int LQMAX, bool LAZY>
__device__ __forceinline__ void dit_lds_from(const Arith<LAZY>& A, u32* buf, int n_el, const PrimeTables& T, int tid,
                                             int nthr) {
  if constexpr (LB > LSTOP) {
    constexpr int LQ = round_lq<LB, LQMAX>();
    dit_lds_from<LB - LQ, LSTOP, LQMAX, LAZY>(A, buf, n_el, T, tid, nthr);
    dit_round_lds<LB, LQ, LAZY>(A, buf, n_el, T, tid, nthr);
    __syncthreads();
  }
}

// log2 of the block size of the last round of a transform of size 2^LB
template <int LB, int LQMAX>
constexpr int last_lb() {
  return LB <= LQMAX ? LB : LQMAX;
}

// The innermost forward round of two buffers, their pointwise product
// (Montgomery, then times sc) and the innermost inverse round, fused: each
// contiguous group of 2^LQL words is read from both buffers by one thread and
// the result written back over the first, so no barrier separates the three
// steps.  Needs a barrier before (the rounds above) and after.
template <int LQL, bool LAZY>
__device__ __forceinline__ void conv_inner(const Arith<LAZY>& A, u32* sa, const u32* sb, int n_el,
                                           const PrimeTables& T, int tid, int nthr, uint2 sc) {
  constexpr int Q = 1 << LQL;
  for (int g = tid; g < (n_el >> LQL); g += nthr) {
    u32 x[Q], y[Q];
    lds_load_contig<Q>(sa, g * Q, x);
    lds_load_contig<Q>(sb, g * Q, y);
    dif_reg<Q>(A, x, T.pf);
    dif_reg<Q>(A, y, T.pf);
#pragma unroll
    for (int t = 0; t < Q; ++t) x[t] = A.mul(A.mont_raw(x[t], y[t]), sc);
    dit_reg<Q>(A, x, T.pi);
    lds_store_contig<Q>(sa, g * Q, x);
  }
}

// ---------------------------------------------------------------------------
// The outermost round of a transform of size B = 2^LB done in registers, for
// a thread that holds x[s] = element tid + (B/Q) s, Q = 2^LQ (the layout of a
// coalesced load by B/Q threads).  Forward: DFT over s, then slot t times
// w_B^{tid rev(t)}; slot t then belongs at position tid + (B/Q) t, the start
// of the Q sub-blocks of size B/Q (the first round of dif_lds, without LDS).
template <int LB, int LQ, bool LAZY>
__device__ __forceinline__ void dif_top_reg(const Arith<LAZY>& A, u32 (&x)[1 << LQ], const PrimeTables& T, int tid) {
  constexpr int Q = 1 << LQ;
  dif_reg<Q, LAZY, true>(A, x, T.pf);
  const uint4* tw = reinterpret_cast<const uint4*>(T.rf[LQ - 1] + (1 << LB) + tid * Q);
#pragma unroll
  for (int k = 0; k < Q / 2; ++k) {
    const uint4 v = cld(tw + k);
    if (k > 0) x[2 * k] = A.mul(x[2 * k], make_uint2(v.x, v.y));
    x[2 * k + 1] = A.mul(x[2 * k + 1], make_uint2(v.z, v.w));
  }
}

// Mirror of dif_top_reg (the last round of dit_lds, unscaled): x[t] holds
// position tid + (B/Q) t; on return x[s] is element tid + (B/Q) s, left in
// [0, 2K) (every caller multiplies it by its untwiddle next).
template <int LB, int LQ, bool LAZY>
__device__ __forceinline__ void dit_top_reg(const Arith<LAZY>& A, u32 (&x)[1 << LQ], const PrimeTables& T, int tid) {
  constexpr int Q = 1 << LQ;
  const uint4* tw = reinterpret_cast<const uint4*>(T.ri[LQ - 1] + (1 << LB) + tid * Q);
#pragma unroll
  for (int k = 0; k < Q / 2; ++k) {
    const uint4 v = cld(tw + k);
    if (k > 0) x[2 * k] = A.mul(x[2 * k], make_uint2(v.x, v.y));
    x[2 * k + 1] = A.mul(x[2 * k + 1], make_uint2(v.z, v.w));
  }
  dit_reg<Q, LAZY, true>(A, x, T.pi);
}

// ---------------------------------------------------------------------------
// Four-step row helpers.  A row of C = 2^LC words is held by NT threads,
// thread tid owning elements tid + NT e (e < EPT = 2^LE, a coalesced load).

// Twiddle element j2 = tid + NT e by g * f[e] (g = w_L^{k1 tid}, f[e] =
// w_L^{k1 NT e}), then the outermost round in registers (dif_top_reg).
template <int LC, int LE, bool LAZY>
__device__ __forceinline__ void row_twist_fwd(const Arith<LAZY>& A, u32 (&x)[1 << LE], uint2 g,
                                              const uint2* __restrict__ f, const PrimeTables& T, int tid) {
#pragma unroll
  for (int e = 0; e < (1 << LE); ++e) x[e] = A.mul(A.mul_raw(x[e], g), cld(f + e));
  dif_top_reg<LC, LE, LAZY>(A, x, T, tid);
}

// The innermost forward round from LDS into registers: x[u Q + t] is slot t
// of the contiguous group tid + nthr u (Q = 2^LQL).
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
