// Three-primes integer product, final steps (section 1): the residues of each
// coefficient modulo p1 = 469762049, p2 = 998244353, p3 = 167772161 give the
// exact coefficient x_k < p1 p2 p3 (Chinese remainder theorem, Garner's
// mixed-radix form); then sum_k x_k 2^{16 k} is written in 16-bit limbs.
//
// Carry propagation: x_k < 2^96 is split into six 16-bit digits and digit d
// is added to limb k + d, so every limb sum s_m = sum_d digit_d(x_{m-d}) is
// below 6 * 2^16.  Limb m is (s_m + carry_m) mod 2^16 and the carry into
// limb m + 1 is (s_m + carry_m) >> 16 <= 6.  A run of limbs maps its carry-in
// c in [0, 7) to a carry-out in [0, 7); these maps are composed with a
// parallel scan (function composition is associative), so the carries of
// all limbs are found in three passes over memory.
#include "internal.h"
#include "trace.h"

namespace pm {

constexpr int kCrtThreads = 256;
constexpr int kCrtPer = 8;                          // limbs per thread
constexpr int kCrtBlock = kCrtThreads * kCrtPer;    // limbs per work-group
constexpr int kCarryStates = 7;                     // carries 0..6

// carry maps packed 3 bits per state: f(c) = (F >> 3c) & 7
__device__ __forceinline__ u32 cm_apply(u32 F, u32 c) { return (F >> (3 * c)) & 7u; }
__device__ __forceinline__ u32 cm_compose(u32 G, u32 F) {  // G after F
  u32 H = 0;
#pragma unroll
  for (u32 c = 0; c < kCarryStates; ++c) H |= cm_apply(G, cm_apply(F, c)) << (3 * c);
  return H;
}
__device__ __forceinline__ u32 cm_identity() {
  u32 H = 0;
#pragma unroll
  for (u32 c = 0; c < kCarryStates; ++c) H |= c << (3 * c);
  return H;
}
// inclusive scan over the work-group: on return maps[t] = F_t o ... o F_0
template <int NT>
__device__ __forceinline__ void cm_block_scan(u32* maps, int tid) {
  for (int off = 1; off < NT; off <<= 1) {
    u32 G = maps[tid];
    if (tid >= off) G = cm_compose(G, maps[tid - off]);
    __syncthreads();
    maps[tid] = G;
    __syncthreads();
  }
}
// map of one limb with sum s
__device__ __forceinline__ u32 cm_limb(u32 s) {
  u32 H = 0;
#pragma unroll
  for (u32 c = 0; c < kCarryStates; ++c) H |= ((s + c) >> 16) << (3 * c);
  return H;
}

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

// x_k as three 32-bit words (x0 least significant)
__device__ __forceinline__ void crt_value(const CrtConsts& K, u32 r1, u32 r2, u32 r3, u32& x0, u32& x1, u32& x2) {
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
  // x = v1 + p1 v2 + p1 p2 v3 < 2^87
  const u64 s = (u64)v1 + (u64)K.p1 * v2;  // < 2^60
  const u64 lo = K.p1p2 * (u64)v3;
  const u64 hi = __umul64hi(K.p1p2, (u64)v3);
  const u64 lo2 = lo + s;
  const u64 hi2 = hi + (lo2 < lo ? 1ull : 0ull);
  x0 = (u32)lo2;
  x1 = (u32)(lo2 >> 32);
  x2 = (u32)hi2;
}

__device__ __forceinline__ u32 digit(u32 x0, u32 x1, u32 x2, int d) {
  const u32 w = d < 2 ? x0 : (d < 4 ? x1 : x2);
  return (d & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Pass 1: limb sums s_m for m < nl and the carry map of each work-group's run.
__global__ void __launch_bounds__(kCrtThreads) k_crt_sums(const u32* __restrict__ r1, const u32* __restrict__ r2,
                                                          const u32* __restrict__ r3, long lc, long nl, CrtConsts K,
                                                          u32* __restrict__ sums, u32* __restrict__ bmap) {
  __shared__ u32 xs[3][kCrtBlock + 8];
  __shared__ u32 maps[kCrtThreads];
  const long m0 = (long)blockIdx.x * kCrtBlock;
  const int tid = threadIdx.x;
  // coefficients k in [m0 - 5, m0 + kCrtBlock)
  for (int i = tid; i < kCrtBlock + 5; i += kCrtThreads) {
    const long k = m0 - 5 + i;
    u32 x0 = 0, x1 = 0, x2 = 0;
    if (k >= 0 && k < lc) crt_value(K, r1[k], r2[k], r3[k], x0, x1, x2);
    xs[0][i] = x0;
    xs[1][i] = x1;
    xs[2][i] = x2;
  }
  __syncthreads();
  u32 F = cm_identity();
  for (int q = 0; q < kCrtPer; ++q) {
    const int i = tid * kCrtPer + q;  // limb m0 + i
    const long m = m0 + i;
    u32 s = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int k = i + 5 - d;  // index of x_{m-d} in xs
      s += digit(xs[0][k], xs[1][k], xs[2][k], d);
    }
    if (m < nl) {
      sums[m] = s;
      F = cm_compose(cm_limb(s), F);
    }
  }
  maps[tid] = F;
  __syncthreads();
  cm_block_scan<kCrtThreads>(maps, tid);
  if (tid == kCrtThreads - 1) bmap[blockIdx.x] = maps[tid];
}

// Pass 2 (one work-group): carry into every run, from the composed maps.
__global__ void __launch_bounds__(1024) k_carry_scan(const u32* __restrict__ bmap, int nblk, u32* __restrict__ cin) {
  __shared__ u32 sc[1024];
  const int tid = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  const int b0 = tid * per;
  u32 F = cm_identity();
  for (int q = 0; q < per; ++q)
    if (b0 + q < nblk) F = cm_compose(bmap[b0 + q], F);
  sc[tid] = F;
  __syncthreads();
  cm_block_scan<1024>(sc, tid);
  u32 c = tid > 0 ? cm_apply(sc[tid - 1], 0) : 0u;
  for (int q = 0; q < per; ++q) {
    if (b0 + q < nblk) {
      cin[b0 + q] = c;
      c = cm_apply(bmap[b0 + q], c);
    }
  }
}

// Pass 3: limbs from the sums and the carries.
__global__ void __launch_bounds__(kCrtThreads) k_carry_apply(const u32* __restrict__ sums, long nl,
                                                             const u32* __restrict__ cin, uint16_t* __restrict__ out) {
  __shared__ u32 maps[kCrtThreads];
  const long m0 = (long)blockIdx.x * kCrtBlock;
  const int tid = threadIdx.x;
  u32 s[kCrtPer];
  u32 F = cm_identity();
#pragma unroll
  for (int q = 0; q < kCrtPer; ++q) {
    const long m = m0 + tid * kCrtPer + q;
    s[q] = m < nl ? sums[m] : 0u;
    F = cm_compose(cm_limb(s[q]), F);
  }
  maps[tid] = F;
  __syncthreads();
  cm_block_scan<kCrtThreads>(maps, tid);
  // carry into this thread's run: the runs of the threads before it
  u32 c = cin[blockIdx.x];
  if (tid > 0) c = cm_apply(maps[tid - 1], c);
#pragma unroll
  for (int q = 0; q < kCrtPer; ++q) {
    const long m = m0 + tid * kCrtPer + q;
    const u32 v = s[q] + c;
    if (m < nl) out[m] = (uint16_t)(v & 0xFFFFu);
    c = v >> 16;
  }
}

size_t crt_workspace_bytes(long nl) {
  const long nblk = (nl + kCrtBlock - 1) / kCrtBlock;
  return (size_t)nl * 4 + (size_t)nblk * 8 + 256;
}

hipError_t launch_crt_carry(const u32* r1, const u32* r2, const u32* r3, long lc, long nl, void* ws, uint16_t* out,
                            hipStream_t s) {
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
  const long nblk = (nl + kCrtBlock - 1) / kCrtBlock;
  u32* sums = (u32*)ws;
  u32* bmap = sums + nl;
  u32* cin = bmap + nblk;
  hipError_t e = launch("crt_sums", k_crt_sums, (unsigned)nblk, kCrtThreads, 0, s, r1, r2, r3, lc, nl, K, sums, bmap);
  if (e == hipSuccess) e = launch("carry_scan", k_carry_scan, 1, 1024, 0, s, bmap, (int)nblk, cin);
  if (e == hipSuccess) e = launch("carry_apply", k_carry_apply, (unsigned)nblk, kCrtThreads, 0, s, sums, nl, cin, out);
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

// The descriptors of the three products, written to device memory so that
// each pass of their common four-step plan runs once over the three primes
// (blockIdx.z selects the prime).
struct JobsOf3 {
  ConvJob j[3];
};

__global__ void k_store_jobs3(JobsOf3 t, ConvJob* __restrict__ out) {
  if (threadIdx.x == 0)
    out[0] = t.j[0];
  else if (threadIdx.x == 1)
    out[1] = t.j[1];
  else if (threadIdx.x == 2)
    out[2] = t.j[2];
}

hipError_t launch_store_jobs3(const ConvJob* jobs, ConvJob* out, hipStream_t s) {
  JobsOf3 t;
  for (int i = 0; i < 3; ++i) t.j[i] = jobs[i];
  return launch("store_jobs", k_store_jobs3, 1, 64, 0, s, t, out);
}

}  // namespace pm
