// Launch dispatch on the prime's value range: every kernel family is compiled
// twice, once per range (LAZY: p < 2^30, values in [0, 2p); CANON: values in
// [0, p)), in separate translation units.
#include "internal.h"

namespace pm {

#define PM_DECL2(name, ...)                  \
  hipError_t name##_lazy0(__VA_ARGS__);      \
  hipError_t name##_lazy1(__VA_ARGS__);

PM_DECL2(launch_lds_conv, const Plan&, const u32*, long, const u32*, long, u32*, long, int, const PrimeTables&, uint2,
         int*, hipStream_t)
PM_DECL2(launch_col_fwd, const Plan&, const void*, long, const void*, long, int, u32*, u32*, int, const PrimeTables&,
         int*, hipStream_t)
PM_DECL2(launch_row_conv, const Plan&, const u32*, const u32*, u32*, int, const PrimeTables&, const RowTables&,
         hipStream_t)
PM_DECL2(launch_col_inv, const Plan&, const u32*, u32*, long, int, const PrimeTables&, hipStream_t)
PM_DECL2(launch_row_xform, const Plan&, const u32*, u32*, long, int, int, const PrimeTables&, const RowTables&,
         hipStream_t)
PM_DECL2(launch_lds_xform, const Plan&, const u32*, long, u32*, long, int, int, int, const PrimeTables&, uint2, int*,
         hipStream_t)
#undef PM_DECL2

hipError_t launch_lds_conv(const Plan& P, const u32* a, long la, const u32* b, long lb, u32* c, long lc, int pidx,
                           const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  return prime_info(pidx).lazy ? launch_lds_conv_lazy1(P, a, la, b, lb, c, lc, pidx, T, sc, err, s)
                               : launch_lds_conv_lazy0(P, a, la, b, lb, c, lc, pidx, T, sc, err, s);
}
hipError_t launch_col_fwd(const Plan& P, const void* a, long za, const void* b, long zb, int in_type, u32* Ta, u32* Tb,
                          int pidx, const PrimeTables& T, int* err, hipStream_t s) {
  return prime_info(pidx).lazy ? launch_col_fwd_lazy1(P, a, za, b, zb, in_type, Ta, Tb, pidx, T, err, s)
                               : launch_col_fwd_lazy0(P, a, za, b, zb, in_type, Ta, Tb, pidx, T, err, s);
}
hipError_t launch_row_conv(const Plan& P, const u32* Ta, const u32* Tb, u32* Tc, int pidx, const PrimeTables& T,
                           const RowTables& W, hipStream_t s) {
  return prime_info(pidx).lazy ? launch_row_conv_lazy1(P, Ta, Tb, Tc, pidx, T, W, s)
                               : launch_row_conv_lazy0(P, Ta, Tb, Tc, pidx, T, W, s);
}
hipError_t launch_col_inv(const Plan& P, const u32* Tc, u32* c, long lc, int pidx, const PrimeTables& T,
                          hipStream_t s) {
  return prime_info(pidx).lazy ? launch_col_inv_lazy1(P, Tc, c, lc, pidx, T, s)
                               : launch_col_inv_lazy0(P, Tc, c, lc, pidx, T, s);
}
hipError_t launch_row_xform(const Plan& P, const u32* in, u32* out, long nout, int dir, int pidx,
                            const PrimeTables& T, const RowTables& W, hipStream_t s) {
  return prime_info(pidx).lazy ? launch_row_xform_lazy1(P, in, out, nout, dir, pidx, T, W, s)
                               : launch_row_xform_lazy0(P, in, out, nout, dir, pidx, T, W, s);
}
hipError_t launch_lds_xform(const Plan& P, const u32* in, long zin, u32* out, long nout, int dir, int natural,
                            int pidx, const PrimeTables& T, uint2 sc, int* err, hipStream_t s) {
  return prime_info(pidx).lazy ? launch_lds_xform_lazy1(P, in, zin, out, nout, dir, natural, pidx, T, sc, err, s)
                               : launch_lds_xform_lazy0(P, in, zin, out, nout, dir, natural, pidx, T, sc, err, s);
}

}  // namespace pm
