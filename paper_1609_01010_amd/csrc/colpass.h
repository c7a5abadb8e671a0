// Column passes of the four-step transforms: rounds of radix at most 16 over
// an [R][W] LDS tile of W adjacent columns (lanes along the columns, so every
// global access is a run of W consecutive words), used by the convolutions'
// column kernels and by the integer product's three-prime kernels.
//
// Split used throughout, for L = R * C: input index j = C j1 + j2 (j1 < R the
// row, j2 < C the column); the column transforms are length-R DIF networks
// (natural in, bit-reversed out), and the rows t < mr are the ones kept.
#pragma once
#include <type_traits>

#include "internal.h"

namespace pm {

// The column tile of an inverse column pass.  Work-groups go to the chip's
// 8 XCDs in turn (linear work-group index mod 8), each XCD with its own L2,
// and a tile of 16 columns reads half of each 128-byte line.  With
// gridDim.x a multiple of 16, work-groups x and x + 8 (one XCD) take tiles
// 2i and 2i + 1 of the same run of 16, so the two halves of a line are read
// through one L2.  Measured: 0.2-2.5 us faster for the inverse passes of the
// 10^6 and integer products; slower (by 2-3 us) for the forward pass of the
// 2^22-point transform, which keeps the plain order.
__device__ __forceinline__ long col_tile_paired() {
  const unsigned x = blockIdx.x, g = gridDim.x;
  return (g & 15u) ? (long)x : (long)(((x >> 4) << 4) | ((x & 7u) << 1) | ((x >> 3) & 1u));
}

// Input element type of the integer product with 32-bit digits: element j
// of the operand is the digit l_{2j} + 2^16 l_{2j+1} of its 16-bit limbs l
// (limbs at or beyond the operand's limb count are zero).  A digit may exceed
// p; it is reduced on load by a Shoup product with the constant 1, which maps
// any 32-bit value into [0, 2p).
struct LimbPair {};

template <typename TIn>
constexpr bool is_limb_pair() {
  return std::is_same<TIn, LimbPair>::value;
}

// radix (log2) of round k (outermost first) of a length-2^LR column transform
template <int LR, int K>
constexpr int col_round_lq() {
  constexpr int seq[11][3] = {{0, 0, 0}, {1, 0, 0}, {2, 0, 0}, {3, 0, 0}, {4, 0, 0}, {2, 3, 0},
                              {3, 3, 0}, {3, 4, 0}, {4, 4, 0}, {3, 3, 3}, {4, 3, 3}};
  return seq[LR][K];
}

// DIF round of radix 2^LQ over the blocks of 2^LB rows that start below mr;
// FROM_GLOBAL: the input is the operand in global memory (rows beyond its
// length z are zero; for LimbPair input z counts limbs), else LDS;
// TO_GLOBAL: output rows below mr go to `out`, else back to LDS
template <int LB, int LQ, bool FROM_GLOBAL, bool TO_GLOBAL, bool LAZY, typename TIn, bool TWIST>
__device__ __forceinline__ void col_dif_round(const Arith<LAZY>& A, u32* sm, int lw, int mr, const PrimeTables& T,
                                              int tid, int nthr, const TIn* __restrict__ in, long z, long C, long col0,
                                              u32* __restrict__ out, const uint2* twf, bool& bad) {
  constexpr int Q = 1 << LQ;
  constexpr int LS = LB - LQ;
  constexpr int K = 16 / Q;
  const int ntask = (((mr + (1 << LB) - 1) >> LB) << LS) << lw;
  // the operand's length in elements, and the constant 1 as a Shoup pair
  // (the digits' reduction)
  const long ze = is_limb_pair<TIn>() ? (z + 1) >> 1 : z;
  uint2 one = make_uint2(0u, 0u);
  if constexpr (FROM_GLOBAL && is_limb_pair<TIn>()) one = cld(T.pf + 1);
  // limb pairs in one 32-bit load when the limbs are 4-byte aligned
  const bool w32 = is_limb_pair<TIn>() && (((uintptr_t)in & 3u) == 0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int task = tid + k * nthr;
    if (task < ntask) {
      const int c = task & ((1 << lw) - 1);
      const int g = task >> lw;
      const int j = g & ((1 << LS) - 1);
      const int base = ((g >> LS) << LB) + j;
      u32 x[Q];
#pragma unroll
      for (int s = 0; s < Q; ++s) {
        const int row = base + (s << LS);
        if constexpr (FROM_GLOBAL && is_limb_pair<TIn>()) {
          const uint16_t* __restrict__ l = (const uint16_t*)in;
          const long i0 = 2 * (C * row + col0 + c);
          u32 d;
          if (w32 && i0 + 1 < z) {
            d = gld((const u32*)l + (i0 >> 1));
          } else {
            const u32 lo = i0 < z ? (u32)gld(l + i0) : 0u;
            const u32 hi = i0 + 1 < z ? (u32)gld(l + i0 + 1) : 0u;
            d = lo | (hi << 16);
          }
          x[s] = A.mul(d, one);
        } else if constexpr (FROM_GLOBAL) {
          const long pos = C * row + col0 + c;
          x[s] = pos < z ? (u32)gld(in + pos) : 0u;
          bad |= x[s] >= A.p;
          if constexpr (TWIST) x[s] = A.mul(x[s], cld(twf + row));
        } else {
          x[s] = sm[(row << lw) + c];
        }
      }
      // the first round spans whole columns (LB = log R): rows R/2 and up
      // are zero when the operand has at most L/2 values
      if (FROM_GLOBAL && (C << (LB - 1)) >= ze)
        dif_reg<Q, LAZY, (LS > 0), true>(A, x, T.pf);
      else
        dif_reg<Q, LAZY, (LS > 0)>(A, x, T.pf);
      const uint2* tw = T.rf[LQ - 1] + (1 << LB) + j * Q;
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const int row = base + (t << LS);
        u32 v = x[t];
        if (LS > 0 && t > 0) v = A.mul(v, cld(tw + t));
        if constexpr (TO_GLOBAL) {
          if (row < mr) gst(out + C * row + col0 + c, v);
        } else {
          sm[(row << lw) + c] = v;
        }
      }
    }
  }
}

// The first round's inputs of a tile (the operand's values, zero beyond
// its length z; a limb pair as its raw 32-bit digit), read once by kernels
// that transform the same tile modulo several primes: task k of the thread
// (as col_dif_round numbers them) holds raw[k][s].
template <int LB, int LQ, typename TIn>
__device__ __forceinline__ void col_first_load(u32 (&raw)[16 >> LQ][1 << LQ], int lw, int mr, int tid, int nthr,
                                               const TIn* __restrict__ in, long z, long C, long col0) {
  constexpr int Q = 1 << LQ;
  constexpr int LS = LB - LQ;
  constexpr int K = 16 / Q;
  const int ntask = (((mr + (1 << LB) - 1) >> LB) << LS) << lw;
  const bool w32 = is_limb_pair<TIn>() && (((uintptr_t)in & 3u) == 0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int task = tid + k * nthr;
    const int c = task & ((1 << lw) - 1);
    const int g = task >> lw;
    const int j = g & ((1 << LS) - 1);
    const int base = ((g >> LS) << LB) + j;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      const int row = base + (s << LS);
      const long pos = C * row + col0 + c;
      u32 d = 0;
      if (task < ntask) {
        if constexpr (is_limb_pair<TIn>()) {
          const uint16_t* __restrict__ l = (const uint16_t*)in;
          const long i0 = 2 * pos;
          if (w32 && i0 + 1 < z) {
            d = gld((const u32*)l + pos);
          } else {
            const u32 lo = i0 < z ? (u32)gld(l + i0) : 0u;
            const u32 hi = i0 + 1 < z ? (u32)gld(l + i0 + 1) : 0u;
            d = lo | (hi << 16);
          }
        } else {
          d = pos < z ? (u32)gld(in + pos) : 0u;
        }
      }
      raw[k][s] = d;
    }
  }
}

// The first DIF round (blocks of 2^LB rows, as col_dif_round's from global
// memory) on values col_first_load read, modulo the prime of A: limb pairs
// reduced by the Shoup product with 1, other inputs taken as they are (they
// must be below p: 16-bit limbs are, for every prime); ze: the operand's
// length in elements.
template <int LB, int LQ, bool TO_GLOBAL, bool LAZY, typename TIn>
__device__ __forceinline__ void col_dif_first_pre(const Arith<LAZY>& A, const u32 (&raw)[16 >> LQ][1 << LQ], u32* sm,
                                                  int lw, int mr, const PrimeTables& T, int tid, int nthr, long ze,
                                                  long C, long col0, u32* __restrict__ out) {
  constexpr int Q = 1 << LQ;
  constexpr int LS = LB - LQ;
  constexpr int K = 16 / Q;
  const int ntask = (((mr + (1 << LB) - 1) >> LB) << LS) << lw;
  uint2 one = make_uint2(0u, 0u);
  if constexpr (is_limb_pair<TIn>()) one = cld(T.pf + 1);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int task = tid + k * nthr;
    if (task < ntask) {
      const int c = task & ((1 << lw) - 1);
      const int g = task >> lw;
      const int j = g & ((1 << LS) - 1);
      const int base = ((g >> LS) << LB) + j;
      u32 x[Q];
#pragma unroll
      for (int s = 0; s < Q; ++s) x[s] = is_limb_pair<TIn>() ? A.mul(raw[k][s], one) : raw[k][s];
      if ((C << (LB - 1)) >= ze)  // rows R/2 and up are zero
        dif_reg<Q, LAZY, (LS > 0), true>(A, x, T.pf);
      else
        dif_reg<Q, LAZY, (LS > 0)>(A, x, T.pf);
      const uint2* tw = T.rf[LQ - 1] + (1 << LB) + j * Q;
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const int row = base + (t << LS);
        u32 v = x[t];
        if (LS > 0 && t > 0) v = A.mul(v, cld(tw + t));
        if constexpr (TO_GLOBAL) {
          if (row < mr) gst(out + C * row + col0 + c, v);
        } else {
          sm[(row << lw) + c] = v;
        }
      }
    }
  }
}

// rounds K.. of the forward column transform on blocks of 2^LB rows; a
// barrier separates consecutive rounds
template <int LR, int K, int LB, bool LAZY, typename TIn, bool TWIST>
__device__ __forceinline__ void col_dif_rounds(const Arith<LAZY>& A, u32* sm, int lw, int mr, const PrimeTables& T,
                                               int tid, int nthr, const TIn* in, long z, long C, long col0, u32* out,
                                               const uint2* twf, bool& bad) {
  constexpr int LQ = col_round_lq<LR, K>();
  constexpr bool first = K == 0;
  constexpr bool last = LB == LQ;
  col_dif_round<LB, LQ, first, last, LAZY, TIn, TWIST>(A, sm, lw, mr, T, tid, nthr, in, z, C, col0, out, twf, bad);
  if constexpr (!last) {
    __syncthreads();
    col_dif_rounds<LR, K + 1, LB - LQ, LAZY, TIn, TWIST>(A, sm, lw, mr, T, tid, nthr, in, z, C, col0, out, twf, bad);
  }
}

// Columns per work-group: 32 (128-byte row segments) unless the tile of R
// rows would exceed 64 KB, and 16 when the grid would otherwise have fewer
// than min_wg work-groups: the chip's 256 compute units, or two per unit for
// the forward pass of a single operand (the transform hooks), whose half
// as many tiles otherwise leave one work-group per unit.
inline int col_lw(int logR, int logC, long groups, long min_wg = 256) {
  int lw = 5;
  if (logR + lw > 14) lw = 14 - logR;
  if (lw > logC) lw = logC;
  while (lw > 4 && (groups << (logC - lw)) < min_wg) --lw;
  return lw;
}
inline int col_threads(int logR, int lw) {
  const int n = 1 << (lw + logR - 4);
  return n < 64 ? 64 : n;
}

// DIT round of radix 2^LQ over the blocks of 2^LB rows below mr (all whole);
// FROM_GLOBAL: the input rows come from `in` (the innermost round), else LDS
template <int LB, int LQ, bool FROM_GLOBAL, bool LAZY>
__device__ __forceinline__ void col_dit_round(const Arith<LAZY>& A, u32* sm, int lw, int mr, const PrimeTables& T,
                                              int tid, int nthr, const u32* __restrict__ in, long C, long col0) {
  constexpr int Q = 1 << LQ;
  constexpr int LS = LB - LQ;
  constexpr int K = 16 / Q;
  const int ntask = ((mr >> LB) << LS) << lw;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int task = tid + k * nthr;
    if (task < ntask) {
      const int c = task & ((1 << lw) - 1);
      const int g = task >> lw;
      const int j = g & ((1 << LS) - 1);
      const int base = ((g >> LS) << LB) + j;
      const uint2* tw = T.ri[LQ - 1] + (1 << LB) + j * Q;
      u32 x[Q];
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const int row = base + (t << LS);
        u32 v = FROM_GLOBAL ? gld(in + C * row + col0 + c) : sm[(row << lw) + c];
        if (LS > 0 && t > 0) v = A.mul(v, cld(tw + t));
        x[t] = v;
      }
      dit_reg<Q>(A, x, T.pi);
#pragma unroll
      for (int s = 0; s < Q; ++s) sm[((base + (s << LS)) << lw) + c] = x[s];
    }
  }
}

// inverse rounds of the length-RB blocks: the mirror of the forward split of
// LRB (rounds K, K-1, .., 0, innermost first); each ends with a barrier
template <int LRB, int K, int LB, bool LAZY>
__device__ __forceinline__ void col_dit_rounds(const Arith<LAZY>& A, u32* sm, int lw, int mr, const PrimeTables& T,
                                               int tid, int nthr, const u32* in, long C, long col0) {
  constexpr int LQ = col_round_lq<LRB, K>();
  if constexpr (LQ > 0) {
    constexpr bool first = LB == 0;
    col_dit_round<LB + LQ, LQ, first, LAZY>(A, sm, lw, mr, T, tid, nthr, in, C, col0);
    __syncthreads();
    if constexpr (K > 0) col_dit_rounds<LRB, K - 1, LB + LQ, LAZY>(A, sm, lw, mr, T, tid, nthr, in, C, col0);
  }
}

template <int LR>
constexpr int col_last_round() {
  return col_round_lq<LR, 2>() ? 2 : (col_round_lq<LR, 1>() ? 1 : 0);
}

// The inverse of radix 32 with M >= 29 known values (inv_column's contract:
// M = 32 unscaled, else scale 1), split over the two lanes of a pair: lane
// `half` holds slots 16 half .. 16 half + 15 (bit-reversed order).  The
// missing values come from the completion matrix, each lane summing over its
// own known values and the partial sums exchanged; the first four levels of
// the network stay within each lane's 16 slots; the last level pairs slot i
// with slot i + 16 across the two lanes.
template <int M, bool LAZY>
__device__ __forceinline__ void inv32_pair(const Arith<LAZY>& A, u32 (&x)[16], int half, const PrimeTables& T) {
  constexpr int D = 32 - M;
  if constexpr (D > 0) {
    const uint2* K = T.kx + fill_offset(5, D);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      u32 acc = 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int k = 16 * half + i;
        if (k < M) acc = A.add(acc, A.mul(x[i], cld(K + r * M + k)));
      }
      acc = A.add(acc, (u32)__shfl_xor((int)acc, 1));
      if (half) x[M - 16 + r] = acc;
    }
  }
  dit_reg<16>(A, x, T.pi);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    // lane 1 forms t = x[i + 16] w_32^-i; lane 0 keeps a = x[i]
    const u32 t = half ? A.mul(x[i], cld(T.pi + 32 + i)) : 0u;
    const u32 recv = (u32)__shfl_xor((int)(half ? t : x[i]), 1);
    x[i] = half ? A.sub(recv, t) : A.add(x[i], recv);
  }
  if constexpr (D > 0) {
    const uint2 qi = cld(T.iv + 5);
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = A.mul(x[i], qi);
  }
}

}  // namespace pm
