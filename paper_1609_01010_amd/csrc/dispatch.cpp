// Launch dispatch on the prime's value range: every kernel family is compiled
// twice, once per range (LAZY: p < 2^30, values in [0, 2p); CANON: values in
// [0, p)), in separate translation units.
#include "internal.h"

namespace pm {

#define PM_DECL2(name, ...)                  \
  hipError_t name##_lazy0(__VA_ARGS__);      \
  hipError_t name##_lazy1(__VA_ARGS__);

PM_DECL2(launch_lds_conv, const Plan&, const JobRef&, int, hipStream_t)
PM_DECL2(launch_col_fwd, const Plan&, int, int, const JobRef&, int, hipStream_t)
PM_DECL2(launch_row_conv, const Plan&, int, const JobRef&, int, hipStream_t)
PM_DECL2(launch_col_inv, const Plan&, const JobRef&, int, hipStream_t)
PM_DECL2(launch_row_xform, const Plan&, const u32*, u32*, long, int, int, const PrimeTables&, const RowTables&,
         hipStream_t)
PM_DECL2(launch_lds_xform, const Plan&, const u32*, long, u32*, long, int, int, int, const PrimeTables&, uint2, int*,
         hipStream_t)
#undef PM_DECL2
hipError_t launch_lds_conv_multi_lazy0(const JobRef&, int, hipStream_t);
hipError_t launch_lds_conv_multi_lazy1(const JobRef&, int, hipStream_t);
bool lds_multi_ok_lazy1(const Plan&);

hipError_t launch_lds_conv_multi(bool lazy, const JobRef& jr, int njobs, hipStream_t s) {
  return lazy ? launch_lds_conv_multi_lazy1(jr, njobs, s) : launch_lds_conv_multi_lazy0(jr, njobs, s);
}
bool lds_multi_ok(const Plan& P) { return lds_multi_ok_lazy1(P); }

hipError_t launch_lds_conv(const Plan& P, bool lazy, const JobRef& jr, int njobs, hipStream_t s) {
  return lazy ? launch_lds_conv_lazy1(P, jr, njobs, s) : launch_lds_conv_lazy0(P, jr, njobs, s);
}
hipError_t launch_col_fwd(const Plan& P, bool lazy, int in_type, int nops, const JobRef& jr, int njobs,
                          hipStream_t s) {
  return lazy ? launch_col_fwd_lazy1(P, in_type, nops, jr, njobs, s)
              : launch_col_fwd_lazy0(P, in_type, nops, jr, njobs, s);
}
hipError_t launch_row_conv(const Plan& P, bool lazy, int max_rows, const JobRef& jr, int njobs, hipStream_t s) {
  return lazy ? launch_row_conv_lazy1(P, max_rows, jr, njobs, s) : launch_row_conv_lazy0(P, max_rows, jr, njobs, s);
}
hipError_t launch_col_inv(const Plan& P, bool lazy, const JobRef& jr, int njobs, hipStream_t s) {
  return lazy ? launch_col_inv_lazy1(P, jr, njobs, s) : launch_col_inv_lazy0(P, jr, njobs, s);
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
