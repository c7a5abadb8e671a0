// Products by their defining sums (Def. 2, eq. 2; and the sums of the two
// quotient rings of eq. 13), for products too small for a transform to pay:
// one thread per output coefficient, exact 64-bit accumulation, one
// reduction per output.
#include "internal.h"
#include "trace.h"

namespace pm {

// ---------------------------------------------------------------------------
// the defining sum c_k = sum_{i+j=k} a_i b_j (Def. 2) for products with < 64
// outputs: one thread per output coefficient

template <bool LAZY>
__global__ void __launch_bounds__(64) k_direct(const u32* __restrict__ a, int la, const u32* __restrict__ b, int lb,
                                              u32* __restrict__ c, ModP mp, int* err) {
  const int k = threadIdx.x;
  const int lc = la + lb - 1;
  if (k >= lc) return;
  u64 acc = 0;  // < 64 terms each below 2^31
  const int i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0;
  const int i1 = k < la - 1 ? k : la - 1;
  for (int i = i0; i <= i1; ++i) {
    const u32 x = a[i], y = b[k - i];
    if (x >= mp.p || y >= mp.p) atomicOr(err, 1);
    acc += (u64)x * y % mp.p;
  }
  c[k] = (u32)(acc % mp.p);
}

// the same over the jobs of a batch: work-group z computes job z's product
// (one thread per output coefficient, at most 64)
__global__ void __launch_bounds__(64) k_direct_jobs(JobRef jr) {
  const ConvJob J = load_job(jr);
  const int k = threadIdx.x;
  const int la = (int)J.la, lb = (int)J.lb;
  if (k >= (int)J.lc) return;
  const u32* __restrict__ a = (const u32*)J.a;
  const u32* __restrict__ b = (const u32*)J.b;
  const u32 p = J.mp.p;
  u64 acc = 0;  // < 64 terms each below 2^31
  const int i0 = k - (lb - 1) > 0 ? k - (lb - 1) : 0;
  const int i1 = k < la - 1 ? k : la - 1;
  bool bad = false;
  for (int i = i0; i <= i1; ++i) {
    const u32 x = gld(a + i), y = gld(b + k - i);
    bad |= x >= p || y >= p;
    acc += (u64)x * y % p;
  }
  if (bad) atomicOr(J.err, 1);
  gst(J.c + k, (u32)(acc % p));
}

// a batch launch's operand and output pointers into its job descriptors:
// job i takes ptrs[3 i], ptrs[3 i + 1], ptrs[3 i + 2] as a, b, c
__global__ void __launch_bounds__(256) k_patch_jobs(ConvJob* jobs, const void* const* ptrs, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  typedef const void* VP;
  PM_GMEM ConvJob* J = (PM_GMEM ConvJob*)(jobs + i);
  const PM_GMEM VP* q = (const PM_GMEM VP*)(ptrs + 3 * (size_t)i);
  J->a = q[0];
  J->b = q[1];
  J->c = (u32*)q[2];
}

// products in Z/pZ[x]/(x^n - 1) (NEG = false, the circular convolution of
// eq. 5) and Z/pZ[x]/(x^n + 1) (NEG = true) by their defining sums, n <= 64:
// c_i = sum_{j+k = i} a_j b_k +- sum_{j+k = i+n} a_j b_k
template <bool NEG>
__global__ void __launch_bounds__(64) k_direct_ring(const u32* __restrict__ a, int la, const u32* __restrict__ b,
                                                   int lb, int n, u32* __restrict__ c, ModP mp, int* err) {
  const int i = threadIdx.x;
  if (i >= n) return;
  u64 pos = 0, neg = 0;  // < 64 terms each below 2^31
  for (int j = 0; j < la; ++j) {
    int k = i - j;
    const bool wrap = k < 0;
    if (wrap) k += n;
    if (k >= lb) continue;
    const u32 x = a[j], y = b[k];
    if (x >= mp.p || y >= mp.p) atomicOr(err, 1);
    const u64 t = (u64)x * y % mp.p;
    if (NEG && wrap)
      neg += t;
    else
      pos += t;
  }
  c[i] = (u32)((pos % mp.p + mp.p - neg % mp.p) % mp.p);
}

hipError_t launch_direct_ring(const u32* a, long la, const u32* b, long lb, long n, bool negacyclic, u32* c, int pidx,
                              int* err, hipStream_t s) {
  const ModP mp = modp_of(prime_info(pidx));
  if (negacyclic) return launch("direct", k_direct_ring<true>, 1, 64, 0, s, a, (int)la, b, (int)lb, (int)n, c, mp, err);
  return launch("direct", k_direct_ring<false>, 1, 64, 0, s, a, (int)la, b, (int)lb, (int)n, c, mp, err);
}

hipError_t launch_patch_jobs(ConvJob* jobs, const void* const* ptrs, int n, hipStream_t s) {
  return launch("patch_jobs", k_patch_jobs, dim3((unsigned)((n + 255) / 256)), 256, 0, s, jobs, ptrs, n);
}

hipError_t launch_direct_jobs(const JobRef& jr, int njobs, hipStream_t s) {
  return launch("direct", k_direct_jobs, dim3(1, 1, njobs), 64, 0, s, jr);
}

hipError_t launch_direct(const u32* a, long la, const u32* b, long lb, u32* c, int pidx, int* err, hipStream_t s) {
  const PrimeInfo& P = prime_info(pidx);
  const ModP mp = modp_of(P);
  if (P.lazy) return launch("direct", k_direct<true>, 1, 64, 0, s, a, (int)la, b, (int)lb, c, mp, err);
  return launch("direct", k_direct<false>, 1, 64, 0, s, a, (int)la, b, (int)lb, c, mp, err);
}

}  // namespace pm
