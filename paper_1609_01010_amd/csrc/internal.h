// Host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <vector>

#include "../../include/polymul.h"
#include "job.h"
#include "ntt_device.h"

namespace pm {

// Raise a kernel's dynamic LDS limit once (the attribute persists; setting it
// on every launch costs host time on the latency-bound small products).
inline void ensure_lds_attr(const void* kern, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(kern);
  if (it != done.end() && it->second >= bytes) return;
  (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  done[kern] = bytes;
}

// the four supported primes p = c * 2^k + 1 with a primitive root g
struct PrimeInfo {
  u32 p;
  u32 g;
  int two_adic;  // k: transform lengths up to 2^k exist
  u32 ninv;      // -p^-1 mod 2^32
  bool lazy;     // p < 2^30: values may live in [0, 2p)
};

int prime_index(u32 p);                 // -1 if unsupported
const PrimeInfo& prime_info(int pidx);  // 0..3
constexpr int kNumPrimes = 4;

// host modular helpers (exact, 64-bit)
u32 h_mulmod(u32 a, u32 b, u32 p);
u32 h_powmod(u32 b, u64 e, u32 p);
u32 h_inv(u32 a, u32 p);
uint2 h_shoup(u32 w, u32 p);  // (w, floor(w 2^32 / p))

struct RowKey {
  int pidx, logL, logC, lnt;
  u32 scale;
  int twist;  // 1: the twisted transform of the nega-circular product
  bool operator<(const RowKey& o) const {
    if (pidx != o.pidx) return pidx < o.pidx;
    if (logL != o.logL) return logL < o.logL;
    if (logC != o.logC) return logC < o.logC;
    if (lnt != o.lnt) return lnt < o.lnt;
    if (scale != o.scale) return scale < o.scale;
    return twist < o.twist;
  }
};

// Device buffers of the cost model's inference, allocated once with the
// device context: plan choice under the learned policy then allocates
// nothing and waits only for its own stream.
constexpr int kMlpInferRows = 8192;  // feature rows per inference launch
struct MlpInfer {
  std::mutex mu;
  hipStream_t s = nullptr;  // the library's inference stream (default priority)
  hipEvent_t ev = nullptr;
  float *dP = nullptr, *dX = nullptr, *dY = nullptr;  // weights, features, outputs (device)
  float *hP = nullptr, *hX = nullptr, *hY = nullptr;  // pinned host staging
  unsigned long ver = 0;                              // model version held in dP (0: none)
};
pm_status mlp_infer_init(MlpInfer* I);
// y[i] = network(X[i]) for B rows of host features, with the weights w of
// model version `ver` (uploaded when it differs from the last one used)
pm_status mlp_infer(MlpInfer* I, const float* w, unsigned long ver, const float* X, int B, float* y);

struct DevCtx {
  int dev = -1;
  MlpInfer infer;
  uint2* prime_mem[kNumPrimes] = {nullptr, nullptr, nullptr, nullptr};
  PrimeTables tabs[kNumPrimes];
  std::map<RowKey, std::pair<uint2*, RowTables>> rowtw;
  int* errflag = nullptr;  // device word: bit 0 = input not reduced
  // workspace per stream: calls on different streams may run concurrently,
  // calls on one stream are ordered by it
  std::map<hipStream_t, std::pair<void*, size_t>> ws;
  // caller-owned workspace per stream (pm_set_workspace): used instead of ws
  std::map<hipStream_t, std::pair<void*, size_t>> user_ws;
  std::mutex mu;
  // the allocation-free product's scratch (a static device array): its
  // address on this device, found once at initialisation (null before)
  u32* scratch = nullptr;
};

DevCtx* ctx_current(pm_status* st);
// the current device's context if it exists (creates nothing)
DevCtx* ctx_lookup();
pm_status ensure_prime_tables(DevCtx* c, int pidx);
// the workspace of stream s, grown to at least `bytes`; a caller-owned one
// (pm_set_workspace) is never grown: PM_ENOMEM if it is smaller
pm_status stream_workspace(DevCtx* c, hipStream_t s, size_t bytes, void** out);
// the workspace stream s uses now (null if none yet)
void* stream_workspace_current(DevCtx* c, hipStream_t s);
// scale: the value multiplied into the inverse factors (1 for none)
pm_status get_row_tables(DevCtx* c, int pidx, int logL, int logC, int lnt, u32 scale, int twist, RowTables* out);
// the same tables written into caller memory `mem` (row_tables_bytes) by
// kernels on stream s, without allocating or waiting
size_t row_tables_bytes(int logL, int logC, int lnt);
pm_status fill_row_tables(int pidx, int logL, int logC, int lnt, u32 scale, int twist, uint2* mem, hipStream_t s,
                          RowTables* out);
// powers psi^(i s) and psi^(-i s), i < L / s, of a primitive 2L-th root of
// unity psi, stride s = 2^log_stride (the nega-circular product's twist)
pm_status get_twist_tables(DevCtx* c, int pidx, int logL, int log_stride, const uint2** fwd, const uint2** inv);

inline ModP modp_of(const PrimeInfo& P) { return ModP{P.p, 2u * P.p, P.ninv}; }

// ---- plans --------------------------------------------------------------
enum PlanKind { PLAN_DIRECT = 0, PLAN_LDS = 1, PLAN_FOURSTEP = 2, PLAN_MIXED = 3 };

struct Plan {
  int kind = PLAN_DIRECT;
  int logL = 0;   // transform length L = 2^logL
  int logRA = 0;  // first (truncated) radix
  int logRB = 0;  // second column radix of the four-step (0: none)
  int logC = 0;   // row length of the four-step
  int ma = 1;     // kept blocks of the first radix, 1..RA
  int lq = 4;     // log radix of the LDS rounds
  int lnt = 0;    // log2 threads of the row pass (0: the default for logC)
  int twist = 0;  // nega-circular product: the passes twist the operands and untwist the result
  int q = 0;      // PLAN_MIXED: the odd factor of the length-q 2^logL circular convolution
};

inline bool same_plan(const Plan& x, const Plan& y) {
  return x.kind == y.kind && x.logL == y.logL && x.logRA == y.logRA && x.logRB == y.logRB && x.logC == y.logC &&
         x.ma == y.ma && x.lq == y.lq && x.lnt == y.lnt && x.twist == y.twist && x.q == y.q;
}

// Timing contexts of the tuner and the cost model: a product on its own
// (latency) or one of many in a batch (throughput, time per product).
constexpr int kCtxSingle = 0;
constexpr int kCtxBatch = 1;

// plan choice (capi.cpp): the cache for (lc, p, context), then the policy
Plan choose_plan(long lc, int pidx, DevCtx* c = nullptr, hipStream_t s = 0, int tctx = kCtxSingle);
void plan_cache_set(long lc, u32 p, const Plan& P, int tctx = kCtxSingle);
bool plan_cache_get(long lc, u32 p, Plan* P, int tctx = kCtxSingle);
// the caller put a plan for (lc, p) into the cache (pm_plan_cache_put)
bool plan_pinned(long lc, u32 p);
// the library's plan without a model or a search
Plan default_plan(long lc, int pidx);
// the tuner's plan space for (lc, prime); with_mixed adds the general-radix
// plans (products on their own only: the batch executor and the cost model
// do not run them)
std::vector<Plan> plan_candidates(long lc, int pidx, bool with_mixed = false);
pm_plan plan_to_pub(const Plan& P);
Plan plan_from_pub(const pm_plan& q);
// workspace bytes a product of output length lc may need, found on the host
size_t product_workspace_bound(long lc, int pidx);
// the cost model's pick (tune.cpp)
Plan learned_plan(long lc, int pidx, bool* ok, int tctx);
// the cost model's picks for the items of one batch, one plan family per
// (transform length, prime); items of at most 64 outputs are left alone
pm_status learned_batch_plans(const std::vector<long>& lcs, const std::vector<int>& pidx, std::vector<Plan>* out);
// the policy in force (capi.cpp)
pm_policy current_policy();
// time every candidate of one length in a context, record the rows, cache the best
pm_status tune_one(DevCtx* c, long lc, int pidx, int reps, hipStream_t s, Plan* best_out, int tctx = kCtxSingle);

// threads of the four-step row pass
inline int plan_row_lnt(const Plan& P) {
  if (P.lnt) return P.lnt;
  return P.logC - 5 < 6 ? 6 : (P.logC - 5 > 9 ? 9 : P.logC - 5);  // 32 elements per thread
}

// relaxed transform length n' = ma * L / RA (q 2^logL for the general radix)
inline long plan_nprime(const Plan& P) {
  return P.kind == PLAN_MIXED ? (long)P.q << P.logL : (long)P.ma << (P.logL - P.logRA);
}

// Fill the job of one product with plan P (capi.cpp).  Ta/Tb: the four-step
// workspace (n' words each) or null; ring 0 the product (or with lc = L the
// circular one), 2 the nega-circular one; rows: the four-step row tables to
// use (null: the context's cached ones, built on first use).
pm_status make_job(DevCtx* c, const Plan& P, int pidx, const void* a, long la, const void* b, long lb, u32* out,
                   long lc, u32* Ta, u32* Tb, ConvJob* J, int ring, const RowTables* rows = nullptr);

// ---- launchers (return hipSuccess or the launch error) --------------------
hipError_t launch_direct(const u32* a, long la, const u32* b, long lb, u32* c, int pidx, int* err, hipStream_t s);
// the defining sums of njobs products of at most 64 outputs (jobs in jr)
hipError_t launch_direct_jobs(const JobRef& jr, int njobs, hipStream_t s);
// jobs[i].a, .b, .c = ptrs[3 i], ptrs[3 i + 1], ptrs[3 i + 2] for i < n (device arrays)
hipError_t launch_patch_jobs(ConvJob* jobs, const void* const* ptrs, int n, hipStream_t s);
constexpr int kKronMaxVars = 8;
hipError_t launch_kron_pack(const u32* a, int nv, const long* da, const long* dc, long n_out, u32* out,
                            hipStream_t s);
hipError_t launch_direct_ring(const u32* a, long la, const u32* b, long lb, long n, bool negacyclic, u32* c, int pidx,
                              int* err, hipStream_t s);
// mixed-radix lengths N = q M (q odd, M a power of two): q in {3, 5, 7, 15, 17}
bool mixed_q_supported(int q);
// x (lx values, zero beyond) -> q rows of M: the length-q transform over j mod q;
// one launch for one operand (x1 null) or two
hipError_t launch_mixed_split(const u32* x0, long lx0, u32* rows0, const u32* x1, long lx1, u32* rows1, int q, long M,
                              int pidx, int* err, hipStream_t s);
// q rows of M -> y_j, j < ly: the inverse length-q transform times q^-1
hipError_t launch_mixed_merge(const u32* rows, int q, long M, u32* y, long ly, int pidx, hipStream_t s);
// q <= 64 job descriptors: base advanced by r * stride (a, b, c) and r * tstride (Ta, Tb)
hipError_t launch_row_jobs(const ConvJob& base, long stride, long tstride, int q, ConvJob* out, hipStream_t s);
// the three jobs (host array) to device memory
// rows[k1][k2] <-> flat[(M k1 + q k2) mod N]
hipError_t launch_mixed_perm(const u32* in, int q, long M, u32* out, int to_flat, hipStream_t s);
// Convolution launches over njobs jobs of one plan class (jobs in jr: the
// single inline job, or a device array indexed by blockIdx.z).
hipError_t launch_lds_conv(const Plan& P, bool lazy, const JobRef& jr, int njobs, hipStream_t s);
// one launch over one-work-group products of several lengths (each job's
// logL and logRA pick its body); lds_multi_ok: the plans it takes
hipError_t launch_lds_conv_multi(bool lazy, const JobRef& jr, int njobs, hipStream_t s);
bool lds_multi_ok(const Plan& P);
// four-step passes; in_type 0 = u32 inputs, 1 = u16; nops = 1 transforms a only
hipError_t launch_col_fwd(const Plan& P, bool lazy, int in_type, int nops, const JobRef& jr, int njobs,
                          hipStream_t s);
hipError_t launch_row_conv(const Plan& P, bool lazy, int max_rows, const JobRef& jr, int njobs, hipStream_t s);
hipError_t launch_col_inv(const Plan& P, bool lazy, const JobRef& jr, int njobs, hipStream_t s);
// standalone row transforms over rows t < ma * RB: dir 0 = twiddle then
// forward (outputs at flat index < nout), dir 1 = inverse then untwiddle and
// multiply by sc
hipError_t launch_row_xform(const Plan& P, const u32* in, u32* out, long nout, int dir, int pidx,
                            const PrimeTables& T, const RowTables& W, hipStream_t s);
// four-step layout (t1 * C + t2 = bit-reversed order) <-> natural order
hipError_t launch_permute(const u32* in, u32* out, int logR, int logC, int to_natural, hipStream_t s);
// one-work-group transform (L <= 2^14) for the hooks: dir 0 forward of zin
// inputs (natural: out[k] = X_k, else out[i] = bit-reversed value, i < nout);
// dir 1 inverse of bit-reversed (or natural) inputs times sc, outputs < nout
hipError_t launch_lds_xform(const Plan& P, const u32* in, long zin, u32* out, long nout, int dir, int natural,
                            int pidx, const PrimeTables& T, uint2 sc, int* err, hipStream_t s);

}  // namespace pm
