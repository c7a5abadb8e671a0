// Kronecker substitution: the dense multivariate product as one univariate
// product (section 1 names multivariate arithmetic among the uses of the
// univariate product).  With the product's box dc[i] = da[i] + db[i] - 1 and
// strides s_i = prod_{j > i} dc[j], exponent vector e maps to sum_i e_i s_i.
// The packed operand holds a[e] there and zero elsewhere; no two monomials of
// the product collide, and the univariate product, in index order, is the
// multivariate product laid out row-major over dc.
#include "internal.h"
#include "trace.h"

namespace pm {

struct KronShape {
  int nv;
  long da[kKronMaxVars];  // the operand's box (1 + degree per variable)
  long dc[kKronMaxVars];  // the product's box
};

// out[t] for t < n_out: the coefficient of the monomial whose Kronecker
// position is t, or 0 if that monomial lies outside the operand's box
__global__ void k_kron_pack(const u32* __restrict__ a, KronShape S, long n_out, u32* __restrict__ out) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n_out; t += (long)gridDim.x * blockDim.x) {
    long rem = t, src = 0, sa = 1;
    bool inside = true;
    for (int i = S.nv - 1; i >= 0; --i) {
      const long e = rem % S.dc[i];
      rem /= S.dc[i];
      inside &= e < S.da[i];
      src += e * sa;
      sa *= S.da[i];
    }
    gst(out + t, inside ? gld(a + src) : 0u);
  }
}

hipError_t launch_kron_pack(const u32* a, int nv, const long* da, const long* dc, long n_out, u32* out,
                            hipStream_t s) {
  KronShape S;
  S.nv = nv;
  for (int i = 0; i < kKronMaxVars; ++i) {
    S.da[i] = i < nv ? da[i] : 1;
    S.dc[i] = i < nv ? dc[i] : 1;
  }
  long blocks = (n_out + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  return launch("kron_pack", k_kron_pack, (unsigned)blocks, 256, 0, s, a, S, n_out, out);
}

}  // namespace pm
