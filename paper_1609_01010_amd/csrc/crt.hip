// Three-primes integer product (section 1): the digit sequences are
// convolved modulo p1 = 469762049, p2 = 998244353, p3 = 167772161, the three
// residues of every coefficient give the exact coefficient x_k < p1 p2 p3
// (Chinese remainder theorem, Garner's mixed-radix form), and sum_k x_k
// 2^{D k} is written in 16-bit limbs.  The digits are the 16-bit limbs
// themselves (D = 16), or pairs of them (D = 32: digit j = l_{2j} + 2^16
// l_{2j+1}), which halves the transform length; with at most 2^21 digits per
// operand (na + nb - 1 <= 2^23 limbs) every x_k < 2^21 (2^32 - 1)^2 < 2^85
// still lies below p1 p2 p3 (about 2^86.02), so it is exact.
//
// When the three primes share one four-step plan, the column passes run once
// for all three: the forward pass reads each tile of limbs once and
// transforms it modulo each prime in turn, and the inverse pass inverts each
// prime's tile in turn, keeps the residues in registers and combines them, so
// only the coefficients x_k reach memory (never the residues).  For the
// supported sizes (na + nb - 1 <= 2^23, so min(na, nb) <= 2^22) every
// x_k < 2^22 (2^16 - 1)^2 < 2^54 fits one 64-bit word.
//
// Carries (D = 16): x_k < 2^54 is four 16-bit digits; digit d goes to limb k + d, so
// the limb sum s_m = sum_{d<4} digit_d(x_{m-d}) < 2^18.  Splitting s_m into
// its low 16 bits and its high part h_m <= 3, the value t_m = lo(s_m) +
// h_{m-1} <= 2^16 + 2 leaves carries of 0 or 1 only: limb m is (t_m + c_m)
// mod 2^16 and c_{m+1} = (t_m + c_m) >> 16.  A run of limbs maps its
// carry-in c in {0, 1} to a carry-out; the maps compose associatively, so
// the carries are a scan, done in two passes: the map of every work-group's
// run (the map of its last limb that does not propagate, so the pass reads
// little more than one chunk of 64 limbs per run), then each work-group takes
// its carry-in from the maps before it and writes its limbs.  With D = 32
// the same scan runs over 32-bit words (below).
#include "colpass.h"
#include "internal.h"
#include "trace.h"

namespace pm {

typedef u64 u64x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Garner's reconstruction

struct CrtConsts {
  u32 p1, p2, p3;
  uint2 inv_p1_mod_p2;     // p1^-1 mod p2 (Shoup pair mod p2)
  uint2 p1_mod_p3;         // p1 mod p3
  uint2 inv_p1p2_mod_p3;   // (p1 p2)^-1 mod p3
  u64 p1p2;                // p1 * p2
};

__device__ __forceinline__ u32 shoup_canon(u32 x, uint2 w, u32 p) {
  u32 r = x * w.x - __umulhi(x, w.y) * p;
  return min(r, r - p);
}

// x = v1 + p1 v2 + p1 p2 v3 from canonical residues r1, r2, r3; the caller
// guarantees x < 2^64 (the sizes the integer product supports)
__device__ __forceinline__ u64 crt_value(const CrtConsts& K, u32 r1, u32 r2, u32 r3) {
  const u32 v1 = r1;
  const u32 v2 = shoup_canon(r2 + K.p2 - v1, K.inv_p1_mod_p2, K.p2);  // v1 < p1 < p2
  u32 v1m3 = v1;
  v1m3 = min(v1m3, v1m3 - K.p3);
  v1m3 = min(v1m3, v1m3 - K.p3);
  v1m3 = min(v1m3, v1m3 - K.p3);  // v1 < p1 < 3 p3
  u32 t = shoup_canon(v2, K.p1_mod_p3, K.p3);  // p1 v2 mod p3
  u32 u = v1m3 + t;
  u = min(u, u - K.p3);
  const u32 v3 = shoup_canon(r3 + K.p3 - u, K.inv_p1p2_mod_p3, K.p3);
  return (u64)v1 + (u64)K.p1 * v2 + K.p1p2 * (u64)v3;
}

// the same value for x < 2^86 (32-bit digits): (low 64 bits, bits 64..)
__device__ __forceinline__ uint4 crt_value_wide(const CrtConsts& K, u32 r1, u32 r2, u32 r3) {
  const u32 v1 = r1;
  const u32 v2 = shoup_canon(r2 + K.p2 - v1, K.inv_p1_mod_p2, K.p2);
  u32 v1m3 = v1;
  v1m3 = min(v1m3, v1m3 - K.p3);
  v1m3 = min(v1m3, v1m3 - K.p3);
  v1m3 = min(v1m3, v1m3 - K.p3);
  u32 t = shoup_canon(v2, K.p1_mod_p3, K.p3);
  u32 u = v1m3 + t;
  u = min(u, u - K.p3);
  const u32 v3 = shoup_canon(r3 + K.p3 - u, K.inv_p1p2_mod_p3, K.p3);
  const u64 low = (u64)v1 + (u64)K.p1 * v2;  // < 2^59
  const u64 plo = K.p1p2 * (u64)v3;          // p1 p2 v3 mod 2^64
  const u64 phi = __umul64hi(K.p1p2, (u64)v3);
  const u64 lo = low + plo;
  const u32 hi = (u32)phi + (lo < plo ? 1u : 0u);
  return make_uint4((u32)lo, (u32)(lo >> 32), hi, 0u);
}

static CrtConsts crt_consts() {
  const PrimeInfo& P1 = prime_info(prime_index(469762049u));
  const PrimeInfo& P2 = prime_info(prime_index(998244353u));
  const PrimeInfo& P3 = prime_info(prime_index(167772161u));
  CrtConsts K;
  K.p1 = P1.p;
  K.p2 = P2.p;
  K.p3 = P3.p;
  K.inv_p1_mod_p2 = h_shoup(h_inv(P1.p % P2.p, P2.p), P2.p);
  K.p1_mod_p3 = h_shoup(P1.p % P3.p, P3.p);
  K.inv_p1p2_mod_p3 = h_shoup(h_inv(h_mulmod(P1.p % P3.p, P2.p % P3.p, P3.p), P3.p), P3.p);
  K.p1p2 = (u64)P1.p * P2.p;
  return K;
}

// the coefficients from three residue arrays (plans that differ per prime)
__global__ void __launch_bounds__(256) k_crt_x(const u32* __restrict__ r1, const u32* __restrict__ r2,
                                               const u32* __restrict__ r3, long lc, CrtConsts K, u64* __restrict__ X) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k < lc) X[k] = crt_value(K, r1[k], r2[k], r3[k]);
}

// ---------------------------------------------------------------------------
// the three primes' column passes (four-step plan shared by the primes; all
// three are below 2^30, so the LAZY value range)

__device__ __forceinline__ ConvJob job_at(const ConvJob* many, int k) {
  ConvJob J;
  const PM_CMEM uint32_t* s = (const PM_CMEM uint32_t*)(many + k);
  uint32_t* d = reinterpret_cast<uint32_t*>(&J);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ConvJob) / 4); ++i) d[i] = s[i];
  return J;
}

// The descriptors of the three products, passed by value to the forward
// column pass, which also writes them to device memory for the row and
// inverse passes (so that each pass of their common plan runs once over the
// three primes, with no launch of its own to store them).
struct JobsOf3 {
  ConvJob j[3];
};

// Forward columns of one operand (blockIdx.y) modulo the three primes
// (t.j[0..2]), one after the other on the same tile of limbs: the tile's
// first-round values are read from memory once, into registers, and each
// prime reduces and transforms them; the stores of one prime drain while the
// next one computes.
template <int LR, typename TIn>
__global__ void __launch_bounds__(1024) k_col_fwd_int3(JobsOf3 t, ConvJob* __restrict__ jobs_out, int logC, int lw) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    jobs_out[0] = t.j[0];
    jobs_out[1] = t.j[1];
    jobs_out[2] = t.j[2];
  }
  extern __shared__ u32 sm[];  // [R][W]
  constexpr int LQ0 = col_round_lq<LR, 0>();
  const int nthr = blockDim.x;
  const long C = 1l << logC;
  const long col0 = (long)blockIdx.x << lw;
  // the operand, its length and the kept rows are the same for the three
  // primes (one plan)
  const TIn* in = (const TIn*)(blockIdx.y ? t.j[0].b : t.j[0].a);
  const long z = blockIdx.y ? t.j[0].lb : t.j[0].la;
  const long ze = is_limb_pair<TIn>() ? (z + 1) >> 1 : z;
  u32 raw[16 >> LQ0][1 << LQ0];
  col_first_load<LR, LQ0, TIn>(raw, lw, t.j[0].rows, threadIdx.x, nthr, in, z, C, col0);
  bool bad = false;
#pragma unroll 1
  for (int pr = 0; pr < 3; ++pr) {
    // the thread index passes through an empty asm each prime, so the
    // compiler cannot hoist every round's addresses out of the loop and
    // hold them in registers across it
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const ConvJob J = t.j[pr];
    const Arith<true> A(J.mp);
    const PrimeTables T = fresh(J.T);
    u32* out = blockIdx.y ? J.Tb : J.Ta;
    col_dif_first_pre<LR, LQ0, LQ0 == LR, true, TIn>(A, raw, sm, lw, J.rows, T, tid, nthr, ze, C, col0, out);
    if constexpr (LQ0 < LR) {
      __syncthreads();
      col_dif_rounds<LR, 1, LR - LQ0, true, TIn, false>(A, sm, lw, J.rows, T, tid, nthr, in, z, C, col0, out,
                                                        nullptr, bad);
    }
    __syncthreads();  // the next prime reuses the tile
  }
}

// Inverse columns modulo the three primes and Garner's reconstruction: each
// prime's length-RB inverses of the tile (the innermost round from its row
// pass output), then per (column, j1b) task the inverse of radix RA with ma
// known values, into registers; the three residues of every output give x_k,
// written as one 64-bit word.  RA <= 16: a thread owns 16 / RA tasks and keeps
// 48 residues, so work-groups are at most 512 threads (16-column tiles at R =
// 512), which leaves each thread up to 256 registers.
// one prime's inverse columns of the tile (jobs[pr]), residues canonical
template <int LRA, int LRB, int TPT>
__device__ __forceinline__ void inv_tile_prime(const ConvJob* jobs, int pr, u32* sm, long C, int lw, long c0, int nthr,
                                               u32 (&res)[TPT][1 << LRA]) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB, R = RA * RB;
  int tid = threadIdx.x;  // through an empty asm per prime: no addresses hoisted across primes
  asm volatile("" : "+v"(tid));
  const ConvJob J = job_at(jobs, pr);
  const Arith<true> A(J.mp);
  const PrimeTables T = fresh(J.T);
  const int ma = J.ma;
  const int W = 1 << lw;
  col_dit_rounds<LRB, col_last_round<LRB>(), 0, true>(A, sm, lw, ma << LRB, T, tid, nthr, J.Ta, C, c0);
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int task = tid + q * nthr;  // < W RB: the grid has exactly W R / 16 threads
    const int cc = task & (W - 1);
    const int j1b = task >> lw;
    const uint2* tw = T.ri[LRA - 1] + R + j1b * RA;
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
    inv_column<RA, true>(A, x, ma, T);
#pragma unroll
    for (int e = 0; e < RA; ++e) res[q][e] = A.canon(x[e]);
  }
  __syncthreads();  // the next prime reuses the tile
}

// WIDE (32-bit digits): x_k is written as four 32-bit words (the low 64
// bits, the bits from 64 on, and 0), else as one 64-bit word.
template <bool WIDE>
__device__ __forceinline__ void crt_store(void* X, long pos, const CrtConsts& K, u32 r1, u32 r2, u32 r3) {
  if constexpr (WIDE) {
    const uint4 v = crt_value_wide(K, r1, r2, r3);
    *((PM_GMEM u32x4*)X + pos) = u32x4{v.x, v.y, v.z, v.w};
  } else {
    gst((u64*)X + pos, crt_value(K, r1, r2, r3));
  }
}

template <int LRA, int LRB, bool WIDE>
__global__ void __launch_bounds__(512) k_col_inv_crt3(const ConvJob* jobs, int logC, int lw, CrtConsts K,
                                                      void* __restrict__ X) {
  constexpr int RA = 1 << LRA, RB = 1 << LRB;
  constexpr int TPT = 16 / RA;
  static_assert(LRA <= 4, "at most one task of 16 values per thread");
  extern __shared__ u32 sm[];  // [R][W]
  const long C = 1l << logC;
  const int W = 1 << lw;
  const long c0 = col_tile_paired() << lw;
  const int nthr = blockDim.x;
  u32 r1[TPT][RA], r2[TPT][RA], r3[TPT][RA];
  inv_tile_prime<LRA, LRB, TPT>(jobs, 0, sm, C, lw, c0, nthr, r1);
  inv_tile_prime<LRA, LRB, TPT>(jobs, 1, sm, C, lw, c0, nthr, r2);
  inv_tile_prime<LRA, LRB, TPT>(jobs, 2, sm, C, lw, c0, nthr, r3);
  const ConvJob J0 = job_at(jobs, 0);
  const int ma = J0.ma;
  const long lc = J0.lc;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int task = tid + q * nthr;
    const int cc = task & (W - 1);
    const int j1b = task >> lw;
#pragma unroll
    for (int e = 0; e < RA; ++e) {
      const long pos = C * (j1b + RB * e) + c0 + cc;
      if (e < ma && pos < lc) crt_store<WIDE>(X, pos, K, r1[q][e], r2[q][e], r3[q][e]);
    }
  }
}

// The first radix 32 (at least 29 of its blocks kept): each task of 32
// values per prime runs on a pair of lanes, 16 values each (inv32_pair), so
// a thread again keeps 48 residues; work-groups of 2 W RB <= 512 threads.
template <int LRB>
__device__ __forceinline__ void inv_tile_prime32(const ConvJob* jobs, int pr, u32* sm, long C, int lw, long c0,
                                                 int nthr, u32 (&res)[16]) {
  constexpr int RA = 32, RB = 1 << LRB, R = RA * RB;
  int tid = threadIdx.x;  // through an empty asm per prime: no addresses hoisted across primes
  asm volatile("" : "+v"(tid));
  const ConvJob J = job_at(jobs, pr);
  const Arith<true> A(J.mp);
  const PrimeTables T = fresh(J.T);
  const int ma = J.ma;
  const int W = 1 << lw;
  col_dit_rounds<LRB, col_last_round<LRB>(), 0, true>(A, sm, lw, ma << LRB, T, tid, nthr, J.Ta, C, c0);
  const int task = tid >> 1, half = tid & 1;
  const int cc = task & (W - 1);
  const int j1b = task >> lw;
  const uint2* tw = T.ri[4] + R + j1b * RA + 16 * half;
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
    case 29: inv32_pair<29, true>(A, x, half, T); break;
    case 30: inv32_pair<30, true>(A, x, half, T); break;
    case 31: inv32_pair<31, true>(A, x, half, T); break;
    default: inv32_pair<32, true>(A, x, half, T); break;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) res[i] = A.canon(x[i]);
  __syncthreads();  // the next prime reuses the tile
}

template <int LRB, bool WIDE>
__global__ void __launch_bounds__(512) k_col_inv_crt3_32(const ConvJob* jobs, int logC, int lw, CrtConsts K,
                                                         void* __restrict__ X) {
  constexpr int RB = 1 << LRB;
  extern __shared__ u32 sm[];  // [R][W]
  const long C = 1l << logC;
  const int W = 1 << lw;
  const long c0 = col_tile_paired() << lw;
  const int nthr = blockDim.x;
  u32 r1[16], r2[16], r3[16];
  inv_tile_prime32<LRB>(jobs, 0, sm, C, lw, c0, nthr, r1);
  inv_tile_prime32<LRB>(jobs, 1, sm, C, lw, c0, nthr, r2);
  inv_tile_prime32<LRB>(jobs, 2, sm, C, lw, c0, nthr, r3);
  const ConvJob J0 = job_at(jobs, 0);
  const int ma = J0.ma;
  const long lc = J0.lc;
  const int tid = threadIdx.x, task = tid >> 1, half = tid & 1;
  const int cc = task & (W - 1);
  const int j1b = task >> lw;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = 16 * half + i;
    const long pos = C * (j1b + RB * e) + c0 + cc;
    if (e < ma && pos < lc) crt_store<WIDE>(X, pos, K, r1[i], r2[i], r3[i]);
  }
}

// the fused passes: four-step plans with the first radix 16 (a thread then
// owns one inverse task of 16 values per prime) and 2^6 .. 2^9 column rows,
// or the first radix 32 with at least 29 blocks kept (a lane pair per task)
// and 2^7 .. 2^10 column rows
bool int3_fused_ok(const Plan& P) {
  if (P.kind != PLAN_FOURSTEP || P.logRB < 2 || P.logRB > 5) return false;
  return P.logRA == 4 || (P.logRA == 5 && P.ma >= 32 - kFillMax);
}

template <int LR, typename TIn>
static hipError_t fwd_int3_lr(const Plan& P, const JobsOf3& t, ConvJob* jobs, hipStream_t s) {
  const int lw = col_lw(LR, P.logC, 2);
  const long C = 1l << P.logC;
  if (C < (1l << lw) || col_threads(LR, lw) > 1024) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (lw + LR)) * sizeof(u32);
  auto kern = k_col_fwd_int3<LR, TIn>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("col_fwd", kern, dim3((unsigned)(C >> lw), 2, 1), col_threads(LR, lw), lds, s, t, jobs, P.logC, lw);
}

template <typename TIn>
static hipError_t fwd_int3_t(const Plan& P, const JobsOf3& t, ConvJob* jobs, hipStream_t s) {
  switch (P.logRA + P.logRB) {
    case 6: return fwd_int3_lr<6, TIn>(P, t, jobs, s);
    case 7: return fwd_int3_lr<7, TIn>(P, t, jobs, s);
    case 8: return fwd_int3_lr<8, TIn>(P, t, jobs, s);
    case 9: return fwd_int3_lr<9, TIn>(P, t, jobs, s);
    case 10: return fwd_int3_lr<10, TIn>(P, t, jobs, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

// host: J, the three descriptors (operand lengths in limbs); jobs, their
// device copy the pass writes; digits32: the transforms' elements are pairs
// of limbs
hipError_t launch_col_fwd_int3(const Plan& P, const ConvJob* J, ConvJob* jobs, bool digits32, hipStream_t s) {
  if (!int3_fused_ok(P)) return hipErrorInvalidValue;
  JobsOf3 t;
  for (int i = 0; i < 3; ++i) t.j[i] = J[i];
  return digits32 ? fwd_int3_t<LimbPair>(P, t, jobs, s) : fwd_int3_t<uint16_t>(P, t, jobs, s);
}

template <int LRA, int LRB, bool WIDE>
static hipError_t inv_crt3_inst(const Plan& P, const ConvJob* jobs, void* X, hipStream_t s) {
  int lw = col_lw(LRA + LRB, P.logC, 1);
  while (lw > 0 && col_threads(LRA + LRB, lw) > 512) --lw;
  const long C = 1l << P.logC;
  // the kernel gives every thread exactly 16 / RA tasks: W R / 16 threads
  if (C < (1l << lw) || col_threads(LRA + LRB, lw) > 512 || 16 * col_threads(LRA + LRB, lw) != (1 << (lw + LRA + LRB)))
    return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (lw + LRA + LRB)) * sizeof(u32);
  auto kern = k_col_inv_crt3<LRA, LRB, WIDE>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("col_inv", kern, dim3((unsigned)(C >> lw), 1, 1), col_threads(LRA + LRB, lw), lds, s, jobs, P.logC,
                lw, crt_consts(), X);
}

template <int LRB, bool WIDE>
static hipError_t inv_crt3_32_inst(const Plan& P, const ConvJob* jobs, void* X, hipStream_t s) {
  int lw = col_lw(5 + LRB, P.logC, 1);
  while (lw > 0 && col_threads(5 + LRB, lw) > 512) --lw;
  const long C = 1l << P.logC;
  // a lane pair per task: 2 W RB threads, which is W R / 16
  const int nthr = col_threads(5 + LRB, lw);
  if (C < (1l << lw) || nthr > 512 || nthr != 2 * ((1 << lw) << LRB)) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << (lw + 5 + LRB)) * sizeof(u32);
  auto kern = k_col_inv_crt3_32<LRB, WIDE>;
  ensure_lds_attr((const void*)kern, lds);
  return launch("col_inv", kern, dim3((unsigned)(C >> lw), 1, 1), nthr, lds, s, jobs, P.logC, lw, crt_consts(), X);
}

template <bool WIDE>
static hipError_t inv_crt3_w(const Plan& P, const ConvJob* jobs, void* X, hipStream_t s) {
  if (P.logRA == 5) {
    switch (P.logRB) {
      case 2: return inv_crt3_32_inst<2, WIDE>(P, jobs, X, s);
      case 3: return inv_crt3_32_inst<3, WIDE>(P, jobs, X, s);
      case 4: return inv_crt3_32_inst<4, WIDE>(P, jobs, X, s);
      case 5: return inv_crt3_32_inst<5, WIDE>(P, jobs, X, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (P.logRB) {
    case 2: return inv_crt3_inst<4, 2, WIDE>(P, jobs, X, s);
    case 3: return inv_crt3_inst<4, 3, WIDE>(P, jobs, X, s);
    case 4: return inv_crt3_inst<4, 4, WIDE>(P, jobs, X, s);
    case 5: return inv_crt3_inst<4, 5, WIDE>(P, jobs, X, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

// X: u64 per coefficient, or (digits32) uint4 per coefficient
hipError_t launch_col_inv_crt3(const Plan& P, const ConvJob* jobs, void* X, bool digits32, hipStream_t s) {
  if (!int3_fused_ok(P)) return hipErrorInvalidValue;
  return digits32 ? inv_crt3_w<true>(P, jobs, X, s) : inv_crt3_w<false>(P, jobs, X, s);
}

hipError_t launch_crt_x(const u32* r1, const u32* r2, const u32* r3, long lc, u64* X, hipStream_t s) {
  return launch("crt", k_crt_x, (unsigned)((lc + 255) / 256), 256, 0, s, r1, r2, r3, lc, crt_consts(), X);
}

// ---------------------------------------------------------------------------
// carries

constexpr int kCarryThreads = 256;
constexpr int kCarryPer = 16;                             // consecutive limbs per thread
constexpr int kCarryBlock = kCarryThreads * kCarryPer;    // limbs per work-group

// The carry map of a run of limbs, bit c = carry-out for carry-in c.  With
// t_m <= 2^16 + 2 every run's map is one of three: kill (0: no carry out),
// propagate (2: the carry in goes out; the identity) or generate (3: a carry
// out whatever comes in), so a composition is the last map of the sequence
// that is not "propagate".
constexpr u32 kCmapIdentity = 2u;
__device__ __forceinline__ u32 cmap_limb(u32 t) { return (t >> 16) | (((t + 1u) >> 16) << 1); }
__device__ __forceinline__ u32 cmap_compose(u32 g, u32 f) { return g == kCmapIdentity ? f : g; }  // g after f
__device__ __forceinline__ u32 cmap_apply(u32 f, u32 c) { return (f >> c) & 1u; }

__device__ __forceinline__ u32 digit16(u64 x, int d) { return (u32)(x >> (16 * d)) & 0xFFFFu; }


// The thread's limbs m = m1 + i, i < kCarryPer: t_m = lo16(s_m) + hi(s_{m-1})
// with s_m = sum_{d<4} digit_d(x_{m-d}) < 2^18 (x_k = 0 outside [0, lc)), so
// that sum_m t_m 2^{16m} = sum_k x_k 2^{16k}.
__device__ __forceinline__ void carry_front(const u64* __restrict__ X, long lc, long m1, u32 (&t)[kCarryPer]) {
  u64 x[kCarryPer + 4];  // x_{m1 - 4 + i}
  if (m1 >= 4 && m1 + kCarryPer <= lc) {
    // m1 is a multiple of 16 and X 256-byte aligned: 16-byte loads
    const PM_GMEM u64x2* p = (const PM_GMEM u64x2*)(X + m1 - 4);
#pragma unroll
    for (int i = 0; i < (kCarryPer + 4) / 2; ++i) {
      const u64x2 v = p[i];
      x[2 * i] = v.x;
      x[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kCarryPer + 4; ++i) {
      const long k = m1 - 4 + i;
      x[i] = (k >= 0 && k < lc) ? gld(X + k) : 0ull;
    }
  }
  u32 sprev = digit16(x[3], 0) + digit16(x[2], 1) + digit16(x[1], 2) + digit16(x[0], 3);  // s_{m1 - 1}
#pragma unroll
  for (int i = 0; i < kCarryPer; ++i) {
    const u32 sv = digit16(x[i + 4], 0) + digit16(x[i + 3], 1) + digit16(x[i + 2], 2) + digit16(x[i + 1], 3);
    t[i] = (sv & 0xFFFFu) + (sprev >> 16);
    sprev = sv;
  }
}

// the map of the thread's run
__device__ __forceinline__ u32 run_map(const u32 (&t)[kCarryPer]) {
  u32 F = kCmapIdentity;
#pragma unroll
  for (int i = 0; i < kCarryPer; ++i) F = cmap_compose(cmap_limb(t[i]), F);
  return F;
}

// The in-order composition of the maps of the lanes below `below` (a lane
// mask) in the wave: the map of the highest such lane that is not the
// identity, else the identity.
__device__ __forceinline__ u32 wave_prefix_map(u32 F, u64 below) {
  const u64 nz = __ballot(F != kCmapIdentity) & below;
  const int src = nz ? 63 - __clzll((long long)nz) : 0;
  const u32 G = __shfl(F, src);
  return nz ? G : kCmapIdentity;
}

// t_m of one limb (as carry_front, for a single m)
__device__ __forceinline__ u32 carry_t_one(const u64* __restrict__ X, long lc, long m) {
  u64 x[5];  // x_{m-4+i}
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const long k = m - 4 + i;
    x[i] = (k >= 0 && k < lc) ? gld(X + k) : 0ull;
  }
  const u32 sv = digit16(x[4], 0) + digit16(x[3], 1) + digit16(x[2], 2) + digit16(x[1], 3);
  const u32 sp = digit16(x[3], 0) + digit16(x[2], 1) + digit16(x[1], 2) + digit16(x[0], 3);
  return (sv & 0xFFFFu) + (sp >> 16);
}

// Pass 1: the carry map of each work-group's run of kCarryBlock limbs, which
// is the map of its last limb that does not propagate.  One wave per run
// looks at 64 limbs at a time from the run's end backwards and stops at the
// first chunk holding such a limb: for most data the last chunk, at worst
// the whole run.
__global__ void __launch_bounds__(64) k_carry_maps(const u64* __restrict__ X, long lc, long nl,
                                                   u32* __restrict__ bmap) {
  const int lane = threadIdx.x;
  const long m0 = (long)blockIdx.x * kCarryBlock;
  const long mend = min(m0 + (long)kCarryBlock, nl);
  u32 B = kCmapIdentity;
  for (long top = mend; top > m0; top -= 64) {
    const long m = top - 64 + lane;
    const u32 F = m >= m0 ? cmap_limb(carry_t_one(X, lc, m)) : kCmapIdentity;
    const u64 nz = __ballot(F != kCmapIdentity);
    if (nz) {
      B = __shfl(F, 63 - __clzll((long long)nz));
      break;
    }
  }
  if (lane == 0) gst(bmap + blockIdx.x, B);
}

// Pass 2: the carry into the work-group (the last map before it that is not
// the identity, applied to carry 0), then the carry into each thread's run,
// and the limbs (t_m + c_m) mod 2^16.  out16: the output is 16-byte aligned.
__global__ void __launch_bounds__(kCarryThreads) k_carry_limbs(const u64* __restrict__ X, long lc, long nl,
                                                               const u32* __restrict__ bmap,
                                                               uint16_t* __restrict__ out, int out16) {
  __shared__ int wlast[kCarryThreads / 64];
  __shared__ u32 wmap[kCarryThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int blk = (int)blockIdx.x;
  // the highest work-group j < blk whose map is not the identity
  int last = -1;
  for (int j = tid; j < blk; j += kCarryThreads)
    if (gld(bmap + j) != kCmapIdentity) last = j;
  for (int off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off));
  const long m1 = (long)blockIdx.x * kCarryBlock + (long)tid * kCarryPer;
  u32 t[kCarryPer];
  carry_front(X, lc, m1, t);
  const u32 F = run_map(t);
  const u32 below = wave_prefix_map(F, (1ull << lane) - 1);  // lanes before this one
  const u32 W = wave_prefix_map(F, ~0ull);                      // the whole wave
  if (lane == 0) {
    wlast[w] = last;
    wmap[w] = W;
  }
  __syncthreads();
  last = wlast[0];
#pragma unroll
  for (int i = 1; i < kCarryThreads / 64; ++i) last = max(last, wlast[i]);
  u32 c = last >= 0 ? cmap_apply(gld(bmap + last), 0) : 0u;
  for (int i = 0; i < w; ++i) c = cmap_apply(wmap[i], c);
  c = cmap_apply(below, c);
  u32 limb[kCarryPer];
#pragma unroll
  for (int i = 0; i < kCarryPer; ++i) {
    const u32 v = t[i] + c;
    limb[i] = v & 0xFFFFu;
    c = v >> 16;
  }
  if (out16 && m1 + kCarryPer <= nl) {
    PM_GMEM u32x4* o = (PM_GMEM u32x4*)(out + m1);
    o[0] = u32x4{limb[0] | limb[1] << 16, limb[2] | limb[3] << 16, limb[4] | limb[5] << 16, limb[6] | limb[7] << 16};
    o[1] = u32x4{limb[8] | limb[9] << 16, limb[10] | limb[11] << 16, limb[12] | limb[13] << 16,
                 limb[14] | limb[15] << 16};
  } else {
#pragma unroll
    for (int i = 0; i < kCarryPer; ++i)
      if (m1 + i < nl) gst(out + m1 + i, (uint16_t)limb[i]);
  }
}

size_t carry_workspace_bytes(long nl) {
  const long nblk = (nl + kCarryBlock - 1) / kCarryBlock;
  return (size_t)nblk * 4 + 256;
}

hipError_t launch_carry(const u64* X, long lc, long nl, void* ws, uint16_t* out, hipStream_t s) {
  const long nblk = (nl + kCarryBlock - 1) / kCarryBlock;
  u32* bmap = (u32*)ws;
  const int out16 = ((uintptr_t)out & 15u) == 0;
  hipError_t e = launch("carry_maps", k_carry_maps, (unsigned)nblk, 64, 0, s, X, lc, nl, bmap);
  if (e == hipSuccess)
    e = launch("carry_limbs", k_carry_limbs, (unsigned)nblk, kCarryThreads, 0, s, X, lc, nl, bmap, out, out16);
  return e;
}

// ---------------------------------------------------------------------------
// carries over 32-bit words (32-bit digits): x_k < 2^85 is three 32-bit
// words w0, w1, w2 (w2 < 2^21), and word w goes to result word k + w, so the
// word sum S_m = w0(x_m) + w1(x_{m-1}) + w2(x_{m-2}) < 2^33 + 2^21.  With
// hi(S) = S >> 32 <= 2, t_m = lo32(S_m) + hi(S_{m-1}) <= 2^32 + 1 again leaves
// carries of 0 or 1: result word m is (t_m + c_m) mod 2^32 (limbs 2m and
// 2m + 1) and c_{m+1} = (t_m + c_m) >> 32.  The carry maps and their scan are
// those of the limbs, with 2^32 in place of 2^16.

__device__ __forceinline__ u32 cmap_word(u64 t) { return (u32)(t >> 32) | ((u32)((t + 1u) >> 32) << 1); }

__device__ __forceinline__ uint4 x4_at(const uint4* __restrict__ X, long lc, long k) {
  if (k < 0 || k >= lc) return make_uint4(0u, 0u, 0u, 0u);
  const PM_GMEM u32x4* q = (const PM_GMEM u32x4*)X + k;
  const u32x4 v = *q;
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ u64 carry_t_one32(const uint4* __restrict__ X, long lc, long m) {
  const uint4 x0 = x4_at(X, lc, m - 3), x1 = x4_at(X, lc, m - 2), x2 = x4_at(X, lc, m - 1), x3 = x4_at(X, lc, m);
  const u64 sv = (u64)x3.x + x2.y + x1.z;
  const u64 sp = (u64)x2.x + x1.y + x0.z;
  return (sv & 0xFFFFFFFFull) + (sp >> 32);
}

// Pass 1 over words: the map of each work-group's run of kCarryBlock words
// (the map of its last word that does not propagate)
__global__ void __launch_bounds__(64) k_carry_maps32(const uint4* __restrict__ X, long lc, long nw,
                                                     u32* __restrict__ bmap) {
  const int lane = threadIdx.x;
  const long m0 = (long)blockIdx.x * kCarryBlock;
  const long mend = min(m0 + (long)kCarryBlock, nw);
  u32 B = kCmapIdentity;
  for (long top = mend; top > m0; top -= 64) {
    const long m = top - 64 + lane;
    const u32 F = m >= m0 ? cmap_word(carry_t_one32(X, lc, m)) : kCmapIdentity;
    const u64 nz = __ballot(F != kCmapIdentity);
    if (nz) {
      B = __shfl(F, 63 - __clzll((long long)nz));
      break;
    }
  }
  if (lane == 0) gst(bmap + blockIdx.x, B);
}

// LDS index of entry j of a work-group's staged coefficients: one pad word
// per 16, so that threads reading runs of 16 consecutive entries (a stride
// of 17 words) hit distinct banks
__device__ __forceinline__ int carry_pad(int j) { return j + (j >> 4); }
constexpr int kCarryStage = kCarryBlock + 3;                   // x_{m0-3} .. x_{m0+4095}
constexpr int kCarryStageLds = kCarryStage + kCarryStage / 16 + 1;

// Pass 2 over words: each work-group's carry-in, each thread's, and the
// words, written as limbs 2m and 2m + 1 below nl.  The work-group's
// coefficients are read once, coalesced, into LDS (their three words in
// three arrays), and each thread forms the t_m of its run from there.
// out16: the output is 16-byte aligned.
__global__ void __launch_bounds__(kCarryThreads) k_carry_limbs32(const uint4* __restrict__ X, long lc, long nw,
                                                                 long nl, const u32* __restrict__ bmap,
                                                                 uint16_t* __restrict__ out, int out16) {
  __shared__ int wlast[kCarryThreads / 64];
  __shared__ u32 wmap[kCarryThreads / 64];
  __shared__ u32 xw[3][kCarryStageLds];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int blk = (int)blockIdx.x;
  const long m0 = (long)blk * kCarryBlock;
  for (int j = tid; j < kCarryStage; j += kCarryThreads) {
    const uint4 v = x4_at(X, lc, m0 - 3 + j);
    const int q = carry_pad(j);
    xw[0][q] = v.x;
    xw[1][q] = v.y;
    xw[2][q] = v.z;
  }
  int last = -1;
  for (int j = tid; j < blk; j += kCarryThreads)
    if (gld(bmap + j) != kCmapIdentity) last = j;
  for (int off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off));
  const long m1 = m0 + (long)tid * kCarryPer;
  __syncthreads();
  // entry j = m - m0 + 3 holds x_m; S_m = w0(x_m) + w1(x_{m-1}) + w2(x_{m-2})
  u64 t[kCarryPer];
  {
    const int j0 = tid * kCarryPer + 3;
    u64 sprev = (u64)xw[0][carry_pad(j0 - 1)] + xw[1][carry_pad(j0 - 2)] + xw[2][carry_pad(j0 - 3)];
#pragma unroll
    for (int i = 0; i < kCarryPer; ++i) {
      const int j = j0 + i;
      const u64 sv = (u64)xw[0][carry_pad(j)] + xw[1][carry_pad(j - 1)] + xw[2][carry_pad(j - 2)];
      t[i] = (sv & 0xFFFFFFFFull) + (sprev >> 32);
      sprev = sv;
    }
  }
  u32 F = kCmapIdentity;
#pragma unroll
  for (int i = 0; i < kCarryPer; ++i) F = cmap_compose(cmap_word(t[i]), F);
  const u32 below = wave_prefix_map(F, (1ull << lane) - 1);
  const u32 W = wave_prefix_map(F, ~0ull);
  if (lane == 0) {
    wlast[w] = last;
    wmap[w] = W;
  }
  __syncthreads();
  last = wlast[0];
#pragma unroll
  for (int i = 1; i < kCarryThreads / 64; ++i) last = max(last, wlast[i]);
  u32 c = last >= 0 ? cmap_apply(gld(bmap + last), 0) : 0u;
  for (int i = 0; i < w; ++i) c = cmap_apply(wmap[i], c);
  c = cmap_apply(below, c);
  u32 word[kCarryPer];
#pragma unroll
  for (int i = 0; i < kCarryPer; ++i) {
    const u64 v = t[i] + c;
    word[i] = (u32)v;
    c = (u32)(v >> 32);
  }
  const long l1 = 2 * m1;  // the thread's first limb
  if (out16 && l1 + 2 * kCarryPer <= nl) {
    PM_GMEM u32x4* o = (PM_GMEM u32x4*)(out + l1);
#pragma unroll
    for (int q = 0; q < kCarryPer / 4; ++q)
      o[q] = u32x4{word[4 * q], word[4 * q + 1], word[4 * q + 2], word[4 * q + 3]};
  } else {
#pragma unroll
    for (int i = 0; i < kCarryPer; ++i) {
      if (l1 + 2 * i < nl) gst(out + l1 + 2 * i, (uint16_t)word[i]);
      if (l1 + 2 * i + 1 < nl) gst(out + l1 + 2 * i + 1, (uint16_t)(word[i] >> 16));
    }
  }
}

// X: dc coefficients as uint4; nl limbs of output
hipError_t launch_carry32(const void* X, long dc, long nl, void* ws, uint16_t* out, hipStream_t s) {
  const long nw = (nl + 1) / 2;
  const long nblk = (nw + kCarryBlock - 1) / kCarryBlock;
  u32* bmap = (u32*)ws;
  const uint4* X4 = (const uint4*)X;
  const int out16 = ((uintptr_t)out & 15u) == 0;
  hipError_t e = launch("carry_maps", k_carry_maps32, (unsigned)nblk, 64, 0, s, X4, dc, nw, bmap);
  if (e == hipSuccess)
    e = launch("carry_limbs", k_carry_limbs32, (unsigned)nblk, kCarryThreads, 0, s, X4, dc, nw, nl, bmap, out, out16);
  return e;
}

// widen 16-bit limbs to 32-bit words (inputs of the one-work-group plans)
__global__ void k_widen(const uint16_t* __restrict__ in, long n, u32* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

hipError_t launch_widen(const uint16_t* in, long n, u32* out, hipStream_t s) {
  return launch("widen", k_widen, (unsigned)((n + 255) / 256), 256, 0, s, in, n, out);
}

}  // namespace pm
