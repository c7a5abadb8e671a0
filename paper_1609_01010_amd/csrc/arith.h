// Modular arithmetic on 32-bit lanes for NTT-friendly primes p = c * 2^k + 1 < 2^31.
//
// The products of the convolution (Def. 2) are computed exactly in Z/pZ.
// Two value ranges are used, chosen per prime at compile time:
//   LAZY  (p < 2^30): values live in [0, 2p); sums in [0, 4p) still fit 32 bits.
//   CANON (p < 2^31): values live in [0, p);  2p < 2^32 but 4p does not.
// Multiplication by a known constant w uses Shoup's precomputed quotient
// wq = floor(w * 2^32 / p): q = mulhi(x, wq), r = x*w - q*p lies in [0, 2p) for
// any 32-bit x.  Products of two variables use Montgomery reduction with
// R = 2^32 (the factor R^-1 is folded into a later constant).
// gfx950: v_mul_lo_u32 issues at full rate, v_mul_hi_u32 at half rate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint32_t u32;
typedef uint64_t u64;

// Address spaces of device memory.  Pointers that reach a kernel inside a job
// descriptor are generic to the compiler, which then emits flat accesses
// (these also hold up waits for LDS results).  Every access to device memory
// names its space instead: gld/gst for data in global memory, cld for the
// twiddle tables, which no kernel writes; wave-uniform reads of those become
// scalar loads.
#define PM_GMEM __attribute__((address_space(1)))
#define PM_CMEM __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  static_assert(__is_arithmetic(T), "scalar types only");
  return *(const PM_GMEM T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  static_assert(__is_arithmetic(T), "scalar types only");
  *(PM_GMEM T*)p = v;
}
__device__ __forceinline__ uint32_t cld(const uint32_t* p) { return *(const PM_CMEM uint32_t*)p; }
__device__ __forceinline__ uint2 cld(const uint2* p) {
  const PM_CMEM uint2* q = (const PM_CMEM uint2*)p;
  return make_uint2(q->x, q->y);
}
__device__ __forceinline__ uint4 cld(const uint4* p) {
  const PM_CMEM uint4* q = (const PM_CMEM uint4*)p;
  return make_uint4(q->x, q->y, q->z, q->w);
}

// Hide a pointer's value from the optimiser: loads through the result are
// neither merged with loads before this point nor hoisted above it.  Used at
// phase boundaries of long kernels so that the table entries held in scalar
// registers are those of one phase only.
template <typename T>
__device__ __forceinline__ const T* fresh(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

struct ModP {
  u32 p;     // the prime
  u32 p2;    // 2p
  u32 ninv;  // -p^-1 mod 2^32 (Montgomery)
};

template <bool LAZY>
struct Arith {
  u32 p, p2, ninv;
  __device__ __forceinline__ explicit Arith(const ModP& m) : p(m.p), p2(m.p2), ninv(m.ninv) {}
  __device__ __forceinline__ Arith(u32 p_, u32 ninv_) : p(p_), p2(2u * p_), ninv(ninv_) {}

  // the additive bound K: values are kept in [0, K)
  __device__ __forceinline__ u32 K() const { return LAZY ? p2 : p; }
  // [0, 2K) -> [0, K): min(x, x - K) works because x - K wraps above x when x < K
  __device__ __forceinline__ u32 red(u32 x) const { return min(x, x - K()); }
  __device__ __forceinline__ u32 add(u32 a, u32 b) const { return red(a + b); }
  __device__ __forceinline__ u32 sub(u32 a, u32 b) const { return red(a - b + K()); }
  // a - b + K in (0, 2K): an input for mul (Shoup accepts any 32-bit value)
  __device__ __forceinline__ u32 subraw(u32 a, u32 b) const { return a - b + K(); }
  // x * w mod p for a constant (w, wq); result in [0, K)
  __device__ __forceinline__ u32 mul(u32 x, u32 w, u32 wq) const {
    u32 q = __umulhi(x, wq);
    u32 r = x * w - q * p;
    return LAZY ? r : min(r, r - p);
  }
  __device__ __forceinline__ u32 mul(u32 x, uint2 wp) const { return mul(x, wp.x, wp.y); }
  // the same, left in [0, 2p): only for a value that is multiplied again
  __device__ __forceinline__ u32 mul_raw(u32 x, uint2 wp) const { return x * wp.x - __umulhi(x, wp.y) * p; }
  // a * b * 2^-32 mod p for a, b in [0, K); result in [0, K)
  __device__ __forceinline__ u32 mont(u32 a, u32 b) const {
    u32 lo = a * b;
    u32 hi = __umulhi(a, b);
    u32 m = lo * ninv;
    u32 t = __umulhi(m, p);
    u32 r = hi + t + (lo != 0u ? 1u : 0u);  // (a*b + m*p) / 2^32 < 2p
    return LAZY ? r : min(r, r - p);
  }
  // the same, left in [0, 2p): only for a value that is multiplied again
  __device__ __forceinline__ u32 mont_raw(u32 a, u32 b) const {
    u32 lo = a * b;
    u32 m = lo * ninv;
    return __umulhi(a, b) + __umulhi(m, p) + (lo != 0u ? 1u : 0u);
  }
  // any value in [0, K) -> canonical [0, p)
  __device__ __forceinline__ u32 canon(u32 x) const { return LAZY ? min(x, x - p) : x; }
};

// Radix-2 butterflies.
// DIF (Gentleman-Sande): (a, b) -> (a + b, (a - b) * w)      natural in, bit-reversed out
// DIT (Cooley-Tukey):    (a, b) -> (a + b * w, a - b * w)    bit-reversed in, natural out
template <bool LAZY>
__device__ __forceinline__ void bfly_dif(const Arith<LAZY>& A, u32& a, u32& b, uint2 w) {
  u32 s = A.add(a, b);
  b = A.mul(A.subraw(a, b), w);
  a = s;
}
template <bool LAZY>
__device__ __forceinline__ void bfly_dif1(const Arith<LAZY>& A, u32& a, u32& b) {
  u32 s = A.add(a, b);
  b = A.sub(a, b);
  a = s;
}
// the same, outputs left in [0, 2K) (a + b and a - b + K): only where both
// are multiplied next (Shoup accepts any 32-bit input)
template <bool LAZY>
__device__ __forceinline__ void bfly_dif1_raw(const Arith<LAZY>& A, u32& a, u32& b) {
  u32 s = a + b;
  b = A.subraw(a, b);
  a = s;
}
template <bool LAZY>
__device__ __forceinline__ void bfly_dit(const Arith<LAZY>& A, u32& a, u32& b, uint2 w) {
  u32 t = A.mul(b, w);
  b = A.sub(a, t);
  a = A.add(a, t);
}
template <bool LAZY>
__device__ __forceinline__ void bfly_dit1(const Arith<LAZY>& A, u32& a, u32& b) {
  u32 t = b;
  b = A.sub(a, t);
  a = A.add(a, t);
}
// DIT butterflies with outputs left in [0, 2K): only where both are
// multiplied next
template <bool LAZY>
__device__ __forceinline__ void bfly_dit_raw(const Arith<LAZY>& A, u32& a, u32& b, uint2 w) {
  u32 t = A.mul(b, w);
  b = A.subraw(a, t);
  a = a + t;
}
template <bool LAZY>
__device__ __forceinline__ void bfly_dit1_raw(const Arith<LAZY>& A, u32& a, u32& b) {
  u32 t = b;
  b = A.subraw(a, t);
  a = a + t;
}

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

__device__ __forceinline__ u32 bitrev_n(u32 x, int bits) { return bits ? (__brev(x) >> (32 - bits)) : 0u; }
