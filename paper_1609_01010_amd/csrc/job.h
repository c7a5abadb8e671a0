// Per-product job descriptor read by the convolution kernels.  A single
// product passes its job by value in the kernel arguments; a batch passes a
// device array indexed by blockIdx.z (one class of equal plans per launch).
#pragma once
#include "ntt_device.h"

// Row-pass twiddles of the four-step split for (L, C, nt threads): element
// j2 = tid + nt e of row k1 is multiplied by gf[k1 nt + tid] * ff[k1 ept + e]
// = w_L^{k1 j2} (forward) or gi[k1 nt + tid] * fi[k1 ept + e] =
// w_L^{-k1 j2} * scale.  Both tables are laid out row after row, so a row's
// threads read them contiguously.
struct RowTables {
  const uint2* gf;
  const uint2* gi;
  const uint2* ff;
  const uint2* fi;
};

struct ConvJob {
  const void* a;   // operand a (u32, or u16 limbs for the integer product)
  const void* b;   // operand b
  long la, lb;     // operand lengths (positions beyond are zero)
  u32* c;          // la + lb - 1 outputs, canonical
  long lc;
  u32* Ta;         // four-step workspace: n' words each
  u32* Tb;
  int ma;          // kept blocks of the first radix
  int rows;        // four-step rows carried: ma * RB
  ModP mp;
  PrimeTables T;
  RowTables W;     // four-step row twiddles (scale folded into fi)
  uint2 sc;        // one-work-group plans: inverse scale (times 2^32)
  int* err;        // device error word
  // nega-circular products (null otherwise): the input twist psi^(s i) and
  // the output untwist psi^(-s i) by row index i of the pass that reads the
  // operands / writes the result (s = C for four-step plans, 1 otherwise)
  const uint2* twf;
  const uint2* twi;
  int logL;        // the plan's transform length and first radix (log2): the
  int logRA;       // one-work-group kernel that runs products of several lengths
};

struct JobRef {
  ConvJob one;
  const ConvJob* many;
};

// the descriptor array is read through the constant space (wave-uniform
// scalar loads); it is never written while kernels run
__device__ __forceinline__ ConvJob load_job(const JobRef& r) {
  if (r.many) {
    static_assert(sizeof(ConvJob) % 4 == 0, "descriptor copied as words");
    ConvJob J;
    const PM_CMEM uint32_t* s = (const PM_CMEM uint32_t*)(r.many + blockIdx.z);
    uint32_t* d = reinterpret_cast<uint32_t*>(&J);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ConvJob) / 4); ++i) d[i] = s[i];
    return J;
  }
  return r.one;
}
