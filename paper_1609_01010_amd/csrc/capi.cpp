// The C ABI (include/polymul.h): argument validation, plan choice, workspace,
// and the launch sequences of the product, the hooks and the integer product.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <tuple>

#include "internal.h"

namespace pm {
bool int3_fused_ok(const Plan& P);
hipError_t launch_col_fwd_int3(const Plan& P, const ConvJob* J, ConvJob* jobs, bool digits32, hipStream_t s);
hipError_t launch_col_inv_crt3(const Plan& P, const ConvJob* jobs, void* X, bool digits32, hipStream_t s);
hipError_t launch_carry32(const void* X, long dc, long nl, void* ws, uint16_t* out, hipStream_t s);
hipError_t launch_crt_x(const u32* r1, const u32* r2, const u32* r3, long lc, u64* X, hipStream_t s);
hipError_t launch_carry(const u64* X, long lc, long nl, void* ws, uint16_t* out, hipStream_t s);
size_t carry_workspace_bytes(long nl);
hipError_t launch_widen(const uint16_t* in, long n, u32* out, hipStream_t s);

// ---------------------------------------------------------------------------
// the allocation-free product's scratch: the four-step workspace (two arrays
// of at most kNoAllocMaxN words) and the row-pass factor tables of its plan.
// One static device array; each device holds its own copy at its own
// address, found by pm_init (hipGetSymbolAddress) and kept in the context.
constexpr long kNoAllocMaxN = 1l << 21;
constexpr size_t kNoAllocWsWords = 2 * (size_t)kNoAllocMaxN;
constexpr size_t kNoAllocRowWords = (size_t)3 << 19;  // 6 MiB: the row tables of any plan with L <= 2^21
constexpr size_t kScratchWords = kNoAllocWsWords + kNoAllocRowWords;
static __device__ __align__(256) u32 scratch[kScratchWords];

// ---------------------------------------------------------------------------
// plans

static int ceil_log2(long x) {
  int l = 0;
  while ((1l << l) < x) ++l;
  return l;
}

static std::mutex g_plan_mu;
static std::atomic<int> g_policy{PM_POLICY_DEFAULT};
static std::atomic<unsigned long> g_plan_epoch{1};

// changes whenever a plan choice could change (policy, cache, model)
unsigned long plan_epoch() { return g_plan_epoch.load(); }
pm_policy current_policy() { return (pm_policy)g_policy.load(); }
void plan_epoch_bump() { g_plan_epoch.fetch_add(1); }
static std::map<std::tuple<long, u32, int>, Plan> g_plan_cache;
static std::set<std::pair<long, u32>> g_plan_pinned;  // (lc, p) put by the caller (pm_plan_cache_put)

bool plan_valid(const Plan& P, long lc, int pidx) {
  const PrimeInfo& PI = prime_info(pidx);
  if (P.lq != 3 && P.lq != 4) return false;
  if (P.kind == PLAN_DIRECT) return lc >= 1 && lc <= 64;
  if (P.kind == PLAN_MIXED)
    return mixed_q_supported(P.q) && (PI.p - 1) % (u32)P.q == 0 && P.logL >= 7 && P.logL <= PI.two_adic &&
           P.logL <= 24 && lc > 64 && plan_nprime(P) >= lc && P.twist == 0;
  if (P.logL < 1 || P.logL > PI.two_adic || P.logL > 24) return false;
  if (P.logRA < 1 || P.logRA > 5 || P.ma < 1 || P.ma > (1 << P.logRA)) return false;
  if (plan_nprime(P) < lc) return false;
  if (P.kind == PLAN_LDS) {
    return P.logL >= 6 && P.logL <= 14 && P.logRA >= 3 && P.logRA <= P.logL && P.logRB == 0 && P.lq == 4;
  }
  if (P.kind == PLAN_FOURSTEP) {
    if (P.logC < 10 || P.logC > 14) return false;
    if (P.logRB < 0 || P.logRB > 5 || (P.logRB > 0 && P.logRA < 4)) return false;
    const int lnt = plan_row_lnt(P);
    if (lnt < 6 || lnt > 10 || P.logC - lnt < 3 || P.logC - lnt > 5) return false;
    if (P.logC - lnt == 3 && P.lq == 4) return false;  // 8 values per thread: innermost radix 8
    return P.logL == P.logRA + P.logRB + P.logC;
  }
  return false;
}

static int kept_blocks(long lc, int logL, int logRA) {
  const long g = 1l << (logL - logRA);  // granularity L / RA
  return (int)((lc + g - 1) / g);
}

Plan default_plan(long lc, int pidx) {
  // measured on MI355X (the tuner's fastest plans for products alone and in
  // batches): up to L = 2^11 one work-group with the first radix 8; for
  // L = 2^12 .. 2^14 the four-step with rows of 2^10 (128 threads) and a
  // single column radix, which spreads a product over L / 2^10 work-groups
  // where one work-group would leave it on a single compute unit; beyond,
  // row length C = L / 256 (at least 2^10, at most 2^13, and at least
  // L / 1024 so that the columns have at most 32 x 32 points), columns split
  // 16 x R/16, 16 elements per row thread, LDS rounds of radix 8 in the
  // rows; truncation with the finest first radix (32) when the output length
  // is not a power of two
  Plan P;
  if (lc <= 64) {
    P.kind = PLAN_DIRECT;
    return P;
  }
  P.logL = ceil_log2(lc);
  const bool pow2 = (lc & (lc - 1)) == 0;
  (void)pidx;
  if (P.logL <= 11) {
    P.kind = PLAN_LDS;
    P.logRA = 3;
  } else if (P.logL <= 14) {
    P.kind = PLAN_FOURSTEP;
    P.logC = 10;
    P.logRA = P.logL - 10;
    P.logRB = 0;
    P.lnt = 7;
    P.lq = 3;
  } else {
    P.kind = PLAN_FOURSTEP;
    P.logC = P.logL - 8 < 10 ? 10 : (P.logL - 8 > 13 ? 13 : P.logL - 8);
    if (P.logL - P.logC > 10) P.logC = P.logL - 10;
    const int logR = P.logL - P.logC;
    if (logR <= 4) {
      P.logRA = logR;
      P.logRB = 0;
    } else {
      // the first radix 32 only where it truncates more finely than 16
      const bool finer = !pow2 && kept_blocks(lc, P.logL, 5) < 2 * kept_blocks(lc, P.logL, 4);
      P.logRA = (finer || logR - 4 > 5) ? 5 : 4;
      P.logRB = logR - P.logRA;
    }
    P.lnt = P.logC - 4 < 6 ? 6 : P.logC - 4;
    P.lq = 3;
  }
  P.ma = kept_blocks(lc, P.logL, P.logRA);
  return P;
}

// candidate plans for the tuner: every valid (kind, C, RA, RB, lq) with and
// without truncation; with_mixed: also the products through the shortest
// circular convolution of length q 2^k >= lc of each odd factor q the
// general-radix product supports (q dividing p - 1), where it is shorter
// than the power-of-two length
std::vector<Plan> plan_candidates(long lc, int pidx, bool with_mixed) {
  std::vector<Plan> out;
  if (lc <= 64) {
    Plan P;
    out.push_back(P);
    return out;
  }
  const int logL = ceil_log2(lc);
  for (int lq = 3; lq <= 4; ++lq) {
    for (int trunc = 1; trunc >= 0; --trunc) {
      if (logL <= 14 && lq == 4) {
        for (int lra = 3; lra <= 5 && lra <= logL; ++lra) {
          Plan P;
          P.kind = PLAN_LDS;
          P.logL = logL;
          P.logRA = lra;
          P.lq = lq;
          P.ma = trunc ? kept_blocks(lc, logL, lra) : (1 << lra);
          if (!trunc && P.ma == kept_blocks(lc, logL, lra)) continue;
          if (plan_valid(P, lc, pidx)) out.push_back(P);
        }
      }
      if (logL >= 12) {
        for (int lc_ = 10; lc_ <= 14; ++lc_) {
          const int lr = logL - lc_;
          if (lr < 1) continue;
          for (int lra = 1; lra <= 5; ++lra) {
            const int lrb = lr - lra;
            if (lrb < 0 || lrb > 5 || (lrb > 0 && lra < 4)) continue;
            for (int lnt = lc_ - 5; lnt <= lc_ - 3; ++lnt) {
              Plan P;
              P.kind = PLAN_FOURSTEP;
              P.logL = logL;
              P.logC = lc_;
              P.logRA = lra;
              P.logRB = lrb;
              P.lq = lq;
              P.lnt = lnt;
              P.ma = trunc ? kept_blocks(lc, logL, lra) : (1 << lra);
              if (!trunc && P.ma == kept_blocks(lc, logL, lra)) continue;
              if (plan_valid(P, lc, pidx)) out.push_back(P);
            }
          }
        }
      }
    }
  }
  if (with_mixed) {
    for (int q : {3, 5, 7, 15, 17}) {
      Plan P;
      P.kind = PLAN_MIXED;
      P.q = q;
      P.logL = 0;
      while (((long)q << P.logL) < lc) ++P.logL;
      if (((long)q << P.logL) < (1l << logL) && plan_valid(P, lc, pidx)) out.push_back(P);
    }
  }
  return out;
}

void plan_cache_set(long lc, u32 p, const Plan& P, int tctx) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plan_cache[std::make_tuple(lc, p, tctx)] = P;
  plan_epoch_bump();
}

bool plan_pinned(long lc, u32 p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return g_plan_pinned.count(std::make_pair(lc, p)) != 0;
}

bool plan_cache_get(long lc, u32 p, Plan* P, int tctx) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plan_cache.find(std::make_tuple(lc, p, tctx));
  if (it == g_plan_cache.end()) return false;
  *P = it->second;
  return true;
}

// The plan cache first (tuned or recorded plans); then the policy: the cost
// model's argmin (cached), the exhaustive search of this length when a
// device context is at hand (the caller holds its lock), or the default.
// tctx: the context the plan runs in (a product alone, or in a batch).
Plan choose_plan(long lc, int pidx, DevCtx* c, hipStream_t s, int tctx) {
  const u32 p = prime_info(pidx).p;
  Plan P;
  if (plan_cache_get(lc, p, &P, tctx)) return P;
  if (lc > 64 && g_policy == PM_POLICY_LEARNED) {
    bool ok = false;
    P = learned_plan(lc, pidx, &ok, tctx);
    if (ok && plan_valid(P, lc, pidx)) {
      plan_cache_set(lc, p, P, tctx);
      return P;
    }
  }
  if (lc > 64 && g_policy == PM_POLICY_EXHAUSTIVE && c) {
    if (tune_one(c, lc, pidx, 5, s, &P, tctx) == PM_OK) return P;
  }
  return default_plan(lc, pidx);
}

pm_plan plan_to_pub(const Plan& P) {
  pm_plan q;
  q.kind = P.kind;
  q.log_l = P.logL;
  q.log_ra = P.logRA;
  q.log_rb = P.logRB;
  q.log_c = P.logC;
  q.ma = P.ma;
  q.lq = P.lq;
  q.lnt = P.lnt;
  q.q = P.q;
  return q;
}
Plan plan_from_pub(const pm_plan& q) {
  Plan P;
  P.kind = q.kind;
  P.logL = q.log_l;
  P.logRA = q.log_ra;
  P.logRB = q.log_rb;
  P.logC = q.log_c;
  P.ma = q.ma;
  P.lq = q.lq;
  P.lnt = q.lnt;
  P.q = q.kind == PLAN_MIXED ? q.q : 0;
  return P;
}

// ---------------------------------------------------------------------------
// execution

static pm_status dev_status(hipError_t e) { return e == hipSuccess ? PM_OK : PM_EDEVICE; }

// scale constant of the inverse: w = inv * 2^32 mod p (the Montgomery factor
// of the pointwise product is folded in)
static uint2 conv_scale(const Plan& P, int pidx) {
  const PrimeInfo& PI = prime_info(pidx);
  long denom;
  const bool full = P.ma == (1 << P.logRA);
  if (P.kind == PLAN_LDS)
    denom = (1l << (P.logL - P.logRA)) * (full ? (1l << P.logRA) : 1l);
  else
    denom = (1l << P.logC) * (1l << P.logRB) * (full ? (1l << P.logRA) : 1l);
  const u32 inv = h_inv((u32)(denom % PI.p), PI.p);
  return h_shoup(h_mulmod(inv, h_powmod(2, 32, PI.p), PI.p), PI.p);
}

// the plan of the q row products of a general-radix product: the length-M
// circular product's default plan (n' = M; from 2^12 on the four-step, so
// that each row spreads over several compute units)
static Plan mixed_row_plan(long M, int pidx) { return default_plan(M, pidx); }

// the general-radix product's workspace: the rows' job descriptors, then A,
// B, C (q rows of M each), then the four-step workspace of every row
static size_t mixed_workspace_bytes(int q, long M, int pidx) {
  const size_t rows_words = (size_t)q * M;
  const size_t job_bytes = (q * sizeof(ConvJob) + 255) / 256 * 256;
  const bool fourstep = M > 64 && mixed_row_plan(M, pidx).kind == PLAN_FOURSTEP;
  return job_bytes + (fourstep ? 5 : 3) * rows_words * sizeof(u32);
}

size_t plan_workspace_bytes(const Plan& P) {
  // (the row plans of a general-radix product do not depend on the prime)
  if (P.kind == PLAN_MIXED) return mixed_workspace_bytes(P.q, 1l << P.logL, 0);
  if (P.kind != PLAN_FOURSTEP) return 0;
  return 2 * (size_t)plan_nprime(P) * sizeof(u32);
}

// Fill the job of one product with plan P (tables are built on first use,
// unless the row tables are given).
pm_status make_job(DevCtx* c, const Plan& P, int pidx, const void* a, long la, const void* b, long lb, u32* out,
                   long lc, u32* Ta, u32* Tb, ConvJob* J, int ring, const RowTables* rows) {
  pm_status st = ensure_prime_tables(c, pidx);
  if (st) return st;
  const PrimeInfo& PI = prime_info(pidx);
  memset(J, 0, sizeof(*J));
  J->a = a;
  J->b = b;
  J->la = la;
  J->lb = lb;
  J->c = out;
  J->lc = lc;
  J->Ta = Ta;
  J->Tb = Tb;
  J->ma = P.ma;
  J->rows = P.ma << P.logRB;
  J->logL = P.logL;
  J->logRA = P.logRA;
  J->mp = modp_of(PI);
  J->T = c->tabs[pidx];
  J->err = c->errflag;
  if (P.kind == PLAN_DIRECT) return PM_OK;
  J->sc = conv_scale(P, pidx);
  if (ring == 2) {
    st = get_twist_tables(c, pidx, P.logL, P.kind == PLAN_FOURSTEP ? P.logC : 0, &J->twf, &J->twi);
    if (st) return st;
  }
  if (P.kind == PLAN_FOURSTEP) {
    if (rows) {
      J->W = *rows;
      return PM_OK;
    }
    return get_row_tables(c, pidx, P.logL, P.logC, plan_row_lnt(P), J->sc.x, ring == 2, &J->W);
  }
  return PM_OK;
}

// Launch the passes of plan P over njobs jobs of one class (same plan, same
// prime range); max_rows bounds J.rows over the jobs.
pm_status launch_class(const Plan& P, bool lazy, int in_type, const JobRef& jr, int njobs, int max_rows,
                       hipStream_t s) {
  hipError_t e;
  if (P.kind == PLAN_DIRECT) {
    if (in_type != 0) return PM_EINVAL;
    e = launch_direct_jobs(jr, njobs, s);
  } else if (P.kind == PLAN_LDS) {
    e = launch_lds_conv(P, lazy, jr, njobs, s);
  } else {
    e = launch_col_fwd(P, lazy, in_type, 2, jr, njobs, s);
    if (e == hipSuccess) e = launch_row_conv(P, lazy, max_rows, jr, njobs, s);
    if (e == hipSuccess) e = launch_col_inv(P, lazy, jr, njobs, s);
  }
  return dev_status(e);
}

static pm_status run_mixed(DevCtx* ctx, int pidx, int q, long M, const u32* a, long la, const u32* b, long lb, u32* c,
                           long lc, void* ws, hipStream_t s);

// run one product with plan P; `ws` has plan_workspace_bytes(P) bytes
pm_status run_product(DevCtx* c, const Plan& P, const void* a, long la, const void* b, long lb, int in_type, u32* out,
                      long lc, int pidx, void* ws, hipStream_t s) {
  if (P.kind == PLAN_MIXED) {
    if (in_type != 0) return PM_EINVAL;
    return run_mixed(c, pidx, P.q, 1l << P.logL, (const u32*)a, la, (const u32*)b, lb, out, lc, ws, s);
  }
  if (P.kind == PLAN_DIRECT) {
    if (in_type != 0) return PM_EINVAL;
    return dev_status(launch_direct((const u32*)a, la, (const u32*)b, lb, out, pidx, c->errflag, s));
  }
  if (P.kind == PLAN_LDS && in_type != 0) return PM_EINVAL;
  u32* Ta = P.kind == PLAN_FOURSTEP ? (u32*)ws : nullptr;
  u32* Tb = Ta ? Ta + plan_nprime(P) : nullptr;
  JobRef jr;
  jr.many = nullptr;
  pm_status st = make_job(c, P, pidx, a, la, b, lb, out, lc, Ta, Tb, &jr.one, 0);
  if (st) return st;
  return launch_class(P, prime_info(pidx).lazy, in_type, jr, 1, jr.one.rows, s);
}

// `rows` circular products of length n (Def. 4, eq. 5): row r of C is
// row r of A times row r of B mod x^n - 1, rows n words apart; P is the plan
// for length n (n' = L = n).  Beyond the defining sums (n <= 64) every pass
// runs once over all rows: `jobs` receives the rows' descriptors (device
// memory, rows entries) and Ta, Tb hold rows * n words each.
static pm_status cyclic_rows(DevCtx* ctx, int pidx, const Plan& P, const u32* A, const u32* B, u32* C, int rows,
                             long n, ConvJob* jobs, u32* Ta, u32* Tb, hipStream_t s) {
  if (n <= 64) {
    for (int r = 0; r < rows; ++r) {
      const long o = (long)r * n;
      const hipError_t e = launch_direct_ring(A + o, n, B + o, n, n, false, C + o, pidx, ctx->errflag, s);
      if (e != hipSuccess) return PM_EDEVICE;
    }
    return PM_OK;
  }
  ConvJob base;
  pm_status st = make_job(ctx, P, pidx, A, n, B, n, C, n, Ta, Tb, &base, 1);
  if (st) return st;
  if (launch_row_jobs(base, n, n, rows, jobs, s) != hipSuccess) return PM_EDEVICE;
  JobRef jr;
  jr.one = base;
  jr.many = jobs;
  return launch_class(P, prime_info(pidx).lazy, 0, jr, rows, base.rows, s);
}

// the plan of the length-n circular product: the plan for output length n,
// which transforms exactly n points (n' = L = n); twist selects the
// nega-circular variant
static pm_status ring_plan(long n, int pidx, DevCtx* ctx, hipStream_t s, int twist, Plan* out) {
  Plan P = choose_plan(n, pidx, ctx, s);
  if (P.kind == PLAN_MIXED) P = default_plan(n, pidx);  // a plan of the linear product only
  if (twist) {
    P.twist = 1;
    if (P.kind == PLAN_LDS) {  // the twisted one-work-group kernels exist for the first radix 16
      P.logRA = 4;
      P.ma = 16;
    }
  }
  if (P.kind == PLAN_DIRECT || !plan_valid(P, n, pidx) || plan_nprime(P) != n) return PM_ETOOLARGE;
  *out = P;
  return PM_OK;
}

// Products mod x^n - 1 (ring 1) and x^n + 1 (ring 2): length-n transforms,
// no padding; the nega-circular twist is carried by the job (make_job).
static pm_status ring_product(int ring, const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, size_t n,
                              uint32_t p, uint32_t* c, void* stream) {
  if (!a || !b || !c || len_a == 0 || len_b == 0 || n < 1 || (n & (n - 1)) || len_a > n || len_b > n)
    return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  const PrimeInfo& PI = prime_info(pidx);
  const int logn = ceil_log2((long)n);
  if (logn + (ring == 2 ? 1 : 0) > PI.two_adic || logn > 24) return PM_ETOOLARGE;
  pm_status st;
  DevCtx* ctx = ctx_current(&st);
  if (!ctx) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  if (n <= 64)
    return dev_status(
        launch_direct_ring(a, (long)len_a, b, (long)len_b, (long)n, ring == 2, c, pidx, ctx->errflag, s));
  Plan P;
  st = ring_plan((long)n, pidx, ctx, s, ring == 2, &P);
  if (st) return st;
  const size_t wsb = plan_workspace_bytes(P);
  void* ws = nullptr;
  if (wsb) {
    st = stream_workspace(ctx, s, wsb, &ws);
    if (st) return st;
  }
  u32* Ta = P.kind == PLAN_FOURSTEP ? (u32*)ws : nullptr;
  u32* Tb = Ta ? Ta + plan_nprime(P) : nullptr;
  JobRef jr;
  jr.many = nullptr;
  st = make_job(ctx, P, pidx, a, (long)len_a, b, (long)len_b, c, (long)n, Ta, Tb, &jr.one, ring);
  if (st) return st;
  return launch_class(P, PI.lazy, 0, jr, 1, jr.one.rows, s);
}


// Product through the length-N = q M circular convolution, q odd: the split
// into q rows (length-q transform over j mod q), q circular products of
// length M, and the merge (inverse length-q transform, factor q^-1) into the
// lc = la + lb - 1 outputs; N >= lc makes the circular product the product.
// ws: mixed_workspace_bytes(q, M) bytes.
static pm_status run_mixed(DevCtx* ctx, int pidx, int q, long M, const u32* a, long la, const u32* b, long lb, u32* c,
                           long lc, void* ws, hipStream_t s) {
  pm_status st = ensure_prime_tables(ctx, pidx);
  if (st) return st;
  const Plan P = mixed_row_plan(M, pidx);
  const size_t rows_words = (size_t)q * M;
  const size_t job_bytes = (q * sizeof(ConvJob) + 255) / 256 * 256;
  const bool fourstep = M > 64 && P.kind == PLAN_FOURSTEP;
  ConvJob* jobs = (ConvJob*)ws;
  u32* A = (u32*)((char*)ws + job_bytes);
  u32* B = A + rows_words;
  u32* C = B + rows_words;
  u32* Ta = fourstep ? C + rows_words : nullptr;
  u32* Tb = fourstep ? Ta + rows_words : nullptr;
  if (launch_mixed_split(a, la, A, b, lb, B, q, M, pidx, ctx->errflag, s) != hipSuccess) return PM_EDEVICE;
  st = cyclic_rows(ctx, pidx, P, A, B, C, q, M, jobs, Ta, Tb, s);
  if (st) return st;
  return dev_status(launch_mixed_merge(C, q, M, c, lc, pidx, s));
}

static pm_status mixed_product(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                               uint32_t q, uint32_t* c, void* stream) {
  if (!a || !b || !c || len_a == 0 || len_b == 0) return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  const PrimeInfo& PI = prime_info(pidx);
  if (!mixed_q_supported((int)q) || (PI.p - 1) % q) return PM_EUNSUPPORTED;
  const long lc = (long)(len_a + len_b - 1);
  long M = 1;
  while ((long)q * M < lc) M <<= 1;
  const int logM = ceil_log2(M);
  if (logM > PI.two_adic || logM > 24) return PM_ETOOLARGE;
  pm_status st;
  DevCtx* ctx = ctx_current(&st);
  if (!ctx) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  st = stream_workspace(ctx, s, mixed_workspace_bytes((int)q, M, pidx), &ws);
  if (st) return st;
  return run_mixed(ctx, pidx, (int)q, M, a, (long)len_a, b, (long)len_b, c, lc, ws, s);
}

// Workspace a product of output length lc may need, on the host alone: under
// the default policy the cached or default plan's; otherwise (the plan is
// picked by the cost model or by timing at call time, and a batch may fall
// back to the default plans) the most any candidate plan needs.
size_t product_workspace_bound(long lc, int pidx) {
  Plan P;
  if (g_policy == PM_POLICY_DEFAULT || plan_pinned(lc, prime_info(pidx).p)) {
    P = choose_plan(lc, pidx);
    return plan_workspace_bytes(P);
  }
  size_t w = plan_workspace_bytes(default_plan(lc, pidx));
  for (const Plan& Q : plan_candidates(lc, pidx, true)) w = std::max(w, plan_workspace_bytes(Q));
  return w;
}

}  // namespace pm

using namespace pm;

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* pm_status_str(pm_status s) {
  switch (s) {
    case PM_OK:
      return "ok";
    case PM_EINVAL:
      return "invalid argument";
    case PM_EUNSUPPORTED:
      return "unsupported modulus";
    case PM_ETOOLARGE:
      return "transform length too large for the modulus";
    case PM_ENOTREDUCED:
      return "input coefficient not reduced modulo p";
    case PM_ENOMEM:
      return "device allocation failed";
    case PM_EDEVICE:
      return "device error";
  }
  return "unknown status";
}

pm_status pm_init(void) {
  // the environment is read once per process; a bad setting fails every pm_init
  static std::once_flag env_once;
  static pm_status env_st = PM_OK;
  std::call_once(env_once, [] { env_st = pm_config_from_env(); });
  if (env_st) return env_st;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < kNumPrimes; ++i) {
    st = ensure_prime_tables(c, i);
    if (st) return st;
  }
  if (!c->scratch) {
    // this device's copy of the static scratch array (the host-side name is
    // only a stand-in: kernels receive this address)
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PM_EDEVICE;
    c->scratch = (u32*)ptr;
  }
  return PM_OK;
}


static pm_status check_product_args(const void* a, size_t la, const void* b, size_t lb, uint32_t p, const void* c,
                                    int* pidx, long* lc) {
  if (!a || !b || !c || la == 0 || lb == 0) return PM_EINVAL;
  if (la > (1ul << 24) || lb > (1ul << 24)) return PM_ETOOLARGE;
  *pidx = prime_index(p);
  if (*pidx < 0) return PM_EUNSUPPORTED;
  *lc = (long)(la + lb - 1);
  const int logL = ceil_log2(*lc);
  const PrimeInfo& PI = prime_info(*pidx);
  if (*lc > 64 && (logL > PI.two_adic || logL > 24)) return PM_ETOOLARGE;
  return PM_OK;
}

static pm_status product_with(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                              uint32_t* c, const Plan* given, void* stream) {
  int pidx;
  long lc;
  pm_status st = check_product_args(a, len_a, b, len_b, p, c, &pidx, &lc);
  if (st) return st;
  DevCtx* ctx = ctx_current(&st);
  if (!ctx) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  Plan P = given ? *given : choose_plan(lc, pidx, ctx, (hipStream_t)stream);
  if (!plan_valid(P, lc, pidx)) return given ? PM_EINVAL : PM_ETOOLARGE;
  const size_t wsb = plan_workspace_bytes(P);
  void* ws = nullptr;
  if (wsb) {
    st = stream_workspace(ctx, (hipStream_t)stream, wsb, &ws);
    if (st) return st;
  }
  return run_product(ctx, P, a, (long)len_a, b, (long)len_b, 0, c, lc, pidx, ws, (hipStream_t)stream);
}

pm_status pm_poly_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p, uint32_t* c,
                      void* stream) {
  return product_with(a, len_a, b, len_b, p, c, nullptr, stream);
}

pm_status pm_poly_mul_noalloc(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                              uint32_t* c, void* stream) {
  int pidx;
  long lc;
  pm_status st = check_product_args(a, len_a, b, len_b, p, c, &pidx, &lc);
  if (st) return st;
  DevCtx* ctx = ctx_lookup();
  if (!ctx || !ctx->scratch) return PM_EINVAL;  // pm_init has not run on this device
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->prime_mem[pidx]) return PM_EINVAL;
  // the cached plan of the length, else the default one: neither the cost
  // model nor the tuner is consulted
  Plan P;
  if (!plan_cache_get(lc, p, &P, kCtxSingle) || P.kind == PLAN_MIXED) P = default_plan(lc, pidx);
  if (!plan_valid(P, lc, pidx)) return PM_ETOOLARGE;
  hipStream_t s = (hipStream_t)stream;
  if (P.kind == PLAN_DIRECT) return dev_status(launch_direct(a, (long)len_a, b, (long)len_b, c, pidx, ctx->errflag, s));
  JobRef jr;
  jr.many = nullptr;
  if (P.kind == PLAN_LDS) {
    st = make_job(ctx, P, pidx, a, (long)len_a, b, (long)len_b, c, lc, nullptr, nullptr, &jr.one, 0, nullptr);
    if (st) return st;
    return launch_class(P, prime_info(pidx).lazy, 0, jr, 1, jr.one.rows, s);
  }
  const long n = plan_nprime(P);
  const int lnt = plan_row_lnt(P);
  if (n > kNoAllocMaxN || row_tables_bytes(P.logL, P.logC, lnt) > kNoAllocRowWords * sizeof(u32)) return PM_ETOOLARGE;
  u32* Ta = ctx->scratch;
  u32* Tb = Ta + n;
  uint2* rmem = (uint2*)(ctx->scratch + kNoAllocWsWords);
  RowTables W;
  st = fill_row_tables(pidx, P.logL, P.logC, lnt, conv_scale(P, pidx).x, 0, rmem, s, &W);
  if (st) return st;
  st = make_job(ctx, P, pidx, a, (long)len_a, b, (long)len_b, c, lc, Ta, Tb, &jr.one, 0, &W);
  if (st) return st;
  return launch_class(P, prime_info(pidx).lazy, 0, jr, 1, jr.one.rows, s);
}

pm_status pm_workspace_query(size_t len_a, size_t len_b, uint32_t p, size_t* bytes) {
  if (!bytes) return PM_EINVAL;
  int pidx;
  long lc;
  const uint32_t one = 1;
  pm_status st = check_product_args(&one, len_a, &one, len_b, p, &one, &pidx, &lc);
  if (st) return st;
  *bytes = product_workspace_bound(lc, pidx);
  return PM_OK;
}

pm_status pm_set_workspace(void* stream, void* ptr, size_t bytes) {
  if (ptr && bytes == 0) return PM_EINVAL;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  hipStream_t s = (hipStream_t)stream;
  if (ptr)
    c->user_ws[s] = std::make_pair(ptr, bytes);
  else
    c->user_ws.erase(s);
  return PM_OK;
}

pm_status pm_poly_mul_multi(const uint32_t* a, const size_t* dims_a, const uint32_t* b, const size_t* dims_b,
                            int nvars, uint32_t p, uint32_t* c, void* stream) {
  if (!a || !b || !c || !dims_a || !dims_b || nvars < 1 || nvars > kKronMaxVars) return PM_EINVAL;
  long da[kKronMaxVars], db[kKronMaxVars], dc[kKronMaxVars];
  long total = 1;
  for (int i = 0; i < nvars; ++i) {
    if (dims_a[i] < 1 || dims_b[i] < 1 || dims_a[i] > (1ul << 24) || dims_b[i] > (1ul << 24)) return PM_EINVAL;
    da[i] = (long)dims_a[i];
    db[i] = (long)dims_b[i];
    dc[i] = da[i] + db[i] - 1;
    total *= dc[i];
    if (total > (1l << 24)) return PM_ETOOLARGE;
  }
  // packed lengths: 1 + sum (d_i - 1) s_i with s_i the product's strides
  long la = 1, lb = 1, stride = 1;
  for (int i = nvars - 1; i >= 0; --i) {
    la += (da[i] - 1) * stride;
    lb += (db[i] - 1) * stride;
    stride *= dc[i];
  }
  int pidx;
  long lc;
  pm_status st = check_product_args(a, (size_t)la, b, (size_t)lb, p, c, &pidx, &lc);
  if (st) return st;
  DevCtx* ctx = ctx_current(&st);
  if (!ctx) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = (hipStream_t)stream;
  const Plan P = choose_plan(lc, pidx, ctx, s);
  if (!plan_valid(P, lc, pidx)) return PM_ETOOLARGE;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t pa = al((size_t)la * 4), pb = al((size_t)lb * 4);
  void* ws = nullptr;
  st = stream_workspace(ctx, s, pa + pb + plan_workspace_bytes(P), &ws);
  if (st) return st;
  u32* ka = (u32*)ws;
  u32* kb = (u32*)((char*)ws + pa);
  hipError_t e = launch_kron_pack(a, nvars, da, dc, la, ka, s);
  if (e == hipSuccess) e = launch_kron_pack(b, nvars, db, dc, lb, kb, s);
  if (e != hipSuccess) return dev_status(e);
  return run_product(ctx, P, ka, la, kb, lb, 0, c, lc, pidx, (char*)ws + pa + pb, s);
}

pm_status pm_cyclic_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, size_t n, uint32_t p,
                        uint32_t* c, void* stream) {
  return ring_product(1, a, len_a, b, len_b, n, p, c, stream);
}

pm_status pm_negacyclic_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, size_t n, uint32_t p,
                            uint32_t* c, void* stream) {
  return ring_product(2, a, len_a, b, len_b, n, p, c, stream);
}

pm_status pm_poly_mul_mixed(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                            uint32_t q, uint32_t* c, void* stream) {
  return mixed_product(a, len_a, b, len_b, p, q, c, stream);
}

pm_status pm_poly_mul_plan(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                           uint32_t* c, const pm_plan* plan, void* stream) {
  if (!plan) return PM_EINVAL;
  Plan P = plan_from_pub(*plan);
  return product_with(a, len_a, b, len_b, p, c, &P, stream);
}

pm_status pm_set_policy(pm_policy policy) {
  if (policy != PM_POLICY_DEFAULT && policy != PM_POLICY_EXHAUSTIVE && policy != PM_POLICY_LEARNED) return PM_EINVAL;
  g_policy.store(policy);
  plan_epoch_bump();
  return PM_OK;
}

pm_policy pm_get_policy(void) { return current_policy(); }

// the plan choice from the process environment: the policy's name is checked
// before anything is applied, then the database and the model are loaded, and
// the policy is set last (a failed load leaves it as it was)
pm_status pm_config_from_env(void) {
  const char* pol = std::getenv("PM_PLAN_POLICY");
  const char* db = std::getenv("PM_TUNE_DB");
  const char* model = std::getenv("PM_MLP_WEIGHTS");
  int policy = -1;
  if (pol && *pol) {
    if (!strcmp(pol, "default"))
      policy = PM_POLICY_DEFAULT;
    else if (!strcmp(pol, "exhaustive"))
      policy = PM_POLICY_EXHAUSTIVE;
    else if (!strcmp(pol, "learned"))
      policy = PM_POLICY_LEARNED;
    else
      return PM_EINVAL;
  }
  pm_status st;
  if (db && *db && (st = pm_tune_db_load(db))) return st;
  if (model && *model && (st = pm_model_load(model))) return st;
  return policy >= 0 ? pm_set_policy((pm_policy)policy) : PM_OK;
}

pm_status pm_plan_for(size_t lc, uint32_t p, pm_plan* plan) { return pm_plan_for_ctx(lc, p, PM_CTX_SINGLE, plan); }

pm_status pm_plan_for_ctx(size_t lc, uint32_t p, int context, pm_plan* plan) {
  if (!plan || lc == 0 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH)) return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  const int logL = ceil_log2((long)lc);
  if (lc > 64 && (logL > prime_info(pidx).two_adic || logL > 24)) return PM_ETOOLARGE;
  *plan = plan_to_pub(choose_plan((long)lc, pidx, nullptr, 0, context));
  return PM_OK;
}

size_t pm_plan_candidates(size_t lc, uint32_t p, pm_plan* out, size_t max_out) {
  const int pidx = prime_index(p);
  if (pidx < 0 || lc == 0) return 0;
  std::vector<Plan> v = plan_candidates((long)lc, pidx, true);
  for (size_t i = 0; i < v.size() && i < max_out && out; ++i) out[i] = plan_to_pub(v[i]);
  return v.size();
}

pm_status pm_plan_cache_put(size_t lc, uint32_t p, const pm_plan* plan) {
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  if (!plan || lc == 0) return PM_EINVAL;
  Plan P = plan_from_pub(*plan);
  if (!plan_valid(P, (long)lc, pidx)) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plan_cache[std::make_tuple((long)lc, p, kCtxSingle)] = P;  // for products alone and in batches
  if (P.kind != PLAN_MIXED) g_plan_cache[std::make_tuple((long)lc, p, kCtxBatch)] = P;
  g_plan_pinned.insert(std::make_pair((long)lc, p));
  plan_epoch_bump();
  return PM_OK;
}

void pm_plan_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plan_cache.clear();
  g_plan_pinned.clear();
  plan_epoch_bump();
}

pm_status pm_stream_check(void* stream) {
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PM_EDEVICE;
  int flag = 0;
  if (hipMemcpy(&flag, c->errflag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return PM_EDEVICE;
  if (flag) {
    if (hipMemset(c->errflag, 0, sizeof(int)) != hipSuccess) return PM_EDEVICE;
    return PM_ENOTREDUCED;
  }
  return PM_OK;
}

// ---- transform hooks --------------------------------------------------------

size_t pm_itft_granularity(size_t L) { return L <= 32 ? 1 : L / 32; }

// the hooks' plan for length L: one work-group up to 2^14, else four-step
// with first radix 32, rows of up to 2^13 (two row work-groups per compute
// unit at 2^22) but at least L / 2^10 (columns of at most 2^10), and 16
// values per row thread
static Plan hook_plan(int logL, int ma) {
  Plan P;
  P.logL = logL;
  if (logL <= 14) {
    P.kind = PLAN_LDS;
    P.logRA = logL < 5 ? logL : 5;
  } else {
    P.kind = PLAN_FOURSTEP;
    P.logRA = 5;
    P.logC = logL - 5 > 13 ? 13 : logL - 5;
    if (logL - P.logC > 10) P.logC = logL - 10;
    P.logRB = logL - 5 - P.logC;
    P.lnt = P.logC - 4;
  }
  P.ma = ma;
  return P;
}

static pm_status hook_setup(size_t L, uint32_t p, int* pidx, int* logL, DevCtx** ctx) {
  if (L < 1 || (L & (L - 1))) return PM_EINVAL;
  *pidx = prime_index(p);
  if (*pidx < 0) return PM_EUNSUPPORTED;
  *logL = ceil_log2((long)L);
  if (*logL > prime_info(*pidx).two_adic || *logL > 24) return PM_ETOOLARGE;
  pm_status st;
  *ctx = ctx_current(&st);
  if (!*ctx) return st;
  return ensure_prime_tables(*ctx, *pidx);
}

// natural-order length-n transform, n = 2^logL >= 2, on an acquired context;
// T: n words of workspace (four-step lengths)
static pm_status ntt_pow2(DevCtx* c, int pidx, int logL, const u32* x, u32* y, long n, int inverse, u32* T,
                          hipStream_t s) {
  const PrimeInfo& PI = prime_info(pidx);
  Plan P = hook_plan(logL, 0);
  P.ma = 1 << P.logRA;
  const uint2 ninv = h_shoup(h_inv((u32)(n % PI.p), PI.p), PI.p);
  if (P.kind == PLAN_LDS)
    return dev_status(
        launch_lds_xform(P, x, n, y, n, inverse ? 1 : 0, 1, pidx, c->tabs[pidx], ninv, c->errflag, s));
  RowTables S;
  pm_status st = get_row_tables(c, pidx, logL, P.logC, plan_row_lnt(P), inverse ? ninv.x : 1u, 0, &S);
  if (st) return st;
  const int logR = P.logRA + P.logRB;
  hipError_t e;
  JobRef jr;
  jr.many = nullptr;
  st = make_job(c, P, pidx, x, n, nullptr, 0, y, n, T, nullptr, &jr.one, 0);
  if (st) return st;
  if (!inverse) {
    e = launch_col_fwd(P, PI.lazy, 0, 1, jr, 1, s);
    if (e == hipSuccess) e = launch_row_xform(P, T, T, n, 0, pidx, c->tabs[pidx], S, s);
    if (e == hipSuccess) e = launch_permute(T, y, logR, P.logC, 1, s);
  } else {
    e = launch_permute(x, T, logR, P.logC, 0, s);
    if (e == hipSuccess) e = launch_row_xform(P, T, T, n, 1, pidx, c->tabs[pidx], S, s);
    if (e == hipSuccess) e = launch_col_inv(P, PI.lazy, jr, 1, s);
  }
  return dev_status(e);
}

// length n = q M, q odd: the prime-factor split into q natural-order
// length-M transforms (mixed.hip states the index maps)
static pm_status ntt_mixed(const uint32_t* x, uint32_t* y, size_t n, uint32_t p, int inverse, void* stream) {
  long M = (long)(n & (~n + 1));  // the largest power of two dividing n
  const int q = (int)(n / (size_t)M);
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  const PrimeInfo& PI = prime_info(pidx);
  if (!mixed_q_supported(q) || (PI.p - 1) % (u32)q) return PM_EUNSUPPORTED;
  const int logM = ceil_log2(M);
  if (logM > PI.two_adic || logM > 24) return PM_ETOOLARGE;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  st = ensure_prime_tables(c, pidx);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  hipStream_t s = (hipStream_t)stream;
  void* wsp = nullptr;
  st = stream_workspace(c, s, (2 * (size_t)n + (size_t)M) * sizeof(u32), &wsp);
  if (st) return st;
  u32* R1 = (u32*)wsp;
  u32* R2 = R1 + n;
  u32* T = R2 + n;
  hipError_t e = inverse ? launch_mixed_perm(x, q, M, R1, 0, s)
                         : launch_mixed_split(x, (long)n, R1, nullptr, 0, nullptr, q, M, pidx, c->errflag, s);
  if (e != hipSuccess) return PM_EDEVICE;
  u32* rows = R1;
  if (M > 1) {
    for (int k1 = 0; k1 < q; ++k1) {
      st = ntt_pow2(c, pidx, logM, R1 + (long)k1 * M, R2 + (long)k1 * M, M, inverse, T, s);
      if (st) return st;
    }
    rows = R2;
  }
  return dev_status(inverse ? launch_mixed_merge(rows, q, M, y, (long)n, pidx, s)
                            : launch_mixed_perm(rows, q, M, y, 1, s));
}

pm_status pm_ntt(const uint32_t* x, uint32_t* y, size_t n, uint32_t p, int inverse, void* stream) {
  if (!x || !y || n < 2) return PM_EINVAL;
  if (n & (n - 1)) return ntt_mixed(x, y, n, p, inverse, stream);
  int pidx, logL;
  DevCtx* c;
  pm_status st = hook_setup(n, p, &pidx, &logL, &c);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  hipStream_t s = (hipStream_t)stream;
  void* wsp = nullptr;
  if (logL > 14) {
    st = stream_workspace(c, s, n * sizeof(u32), &wsp);
    if (st) return st;
  }
  return ntt_pow2(c, pidx, logL, x, y, (long)n, inverse, (u32*)wsp, s);
}

pm_status pm_tft(const uint32_t* x, size_t z, size_t L, size_t n, uint32_t p, uint32_t* out, void* stream) {
  if (!x || !out || z < 1 || n < 1 || z > L || n > L) return PM_EINVAL;
  int pidx, logL;
  DevCtx* c;
  pm_status st = hook_setup(L, p, &pidx, &logL, &c);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  hipStream_t s = (hipStream_t)stream;
  Plan P = hook_plan(logL, 0);
  P.ma = kept_blocks((long)n, logL, P.logRA);
  const uint2 one = h_shoup(1, prime_info(pidx).p);
  if (P.kind == PLAN_LDS)
    return dev_status(
        launch_lds_xform(P, x, (long)z, out, (long)n, 0, 0, pidx, c->tabs[pidx], one, c->errflag, s));
  void* wsp = nullptr;
  st = stream_workspace(c, s, (size_t)plan_nprime(P) * sizeof(u32), &wsp);
  if (st) return st;
  RowTables S;
  st = get_row_tables(c, pidx, logL, P.logC, plan_row_lnt(P), 1u, 0, &S);
  if (st) return st;
  u32* T = (u32*)wsp;
  JobRef jr;
  jr.many = nullptr;
  st = make_job(c, P, pidx, x, (long)z, nullptr, 0, out, (long)n, T, nullptr, &jr.one, 0);
  if (st) return st;
  hipError_t e = launch_col_fwd(P, prime_info(pidx).lazy, 0, 1, jr, 1, s);
  if (e == hipSuccess) e = launch_row_xform(P, T, out, (long)n, 0, pidx, c->tabs[pidx], S, s);
  return dev_status(e);
}

pm_status pm_itft(const uint32_t* v, size_t L, size_t n, uint32_t p, uint32_t* out, void* stream) {
  if (!v || !out || n < 1 || n > L || (L & (L - 1)) || n % pm_itft_granularity(L)) return PM_EINVAL;
  int pidx, logL;
  DevCtx* c;
  pm_status st = hook_setup(L, p, &pidx, &logL, &c);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  const PrimeInfo& PI = prime_info(pidx);
  hipStream_t s = (hipStream_t)stream;
  Plan P = hook_plan(logL, 0);
  P.ma = kept_blocks((long)n, logL, P.logRA);
  const bool full = P.ma == (1 << P.logRA);
  // L u = (unscaled inverse) * L / (length of the unscaled part)
  const uint2 sc = h_shoup(full ? 1u : (u32)(1u << P.logRA), PI.p);
  if (P.kind == PLAN_LDS)
    return dev_status(launch_lds_xform(P, v, (long)n, out, (long)n, 1, 0, pidx, c->tabs[pidx], sc, c->errflag, s));
  void* wsp = nullptr;
  st = stream_workspace(c, s, (size_t)plan_nprime(P) * sizeof(u32), &wsp);
  if (st) return st;
  RowTables S;
  st = get_row_tables(c, pidx, logL, P.logC, plan_row_lnt(P), sc.x, 0, &S);
  if (st) return st;
  u32* T = (u32*)wsp;
  JobRef jr;
  jr.many = nullptr;
  st = make_job(c, P, pidx, v, (long)n, nullptr, 0, out, (long)n, T, nullptr, &jr.one, 0);
  if (st) return st;
  hipError_t e = launch_row_xform(P, v, T, (long)n, 1, pidx, c->tabs[pidx], S, s);
  if (e == hipSuccess) e = launch_col_inv(P, prime_info(pidx).lazy, jr, 1, s);
  return dev_status(e);
}

// ---- three-primes integer product -----------------------------------------------

static const u32 kIntPrimes[3] = {469762049u, 998244353u, 167772161u};

// The integer product's plans and workspace.  When the three primes share
// one four-step plan whose column passes have a fused three-prime form, the
// passes run once over the three primes (the forward columns read the limbs
// once; the inverse columns combine the residues in registers and write the
// coefficients x_k as 64-bit words): the workspace holds each prime's Ta/Tb,
// their descriptors, x and the carry state.  Otherwise each prime's product
// writes a residue array (widened 32-bit operands for plans that need them),
// a kernel combines the residues into x, and the carries follow.
// With 32-bit digits (pairs of limbs; only in the fused form) the
// transforms have da + db - 1 elements (da = ceil(na / 2)), x_k takes 16
// bytes and the carries run over 32-bit words.
struct IntLayout {
  Plan plans[3];
  bool widen = false;
  bool fused = false;
  bool d32 = false;
  long lc = 0;  // coefficients: na + nb - 1, or da + db - 1 with 32-bit digits
  size_t res_b = 0, wid_b = 0, pw = 0, jobs_b = 0, x_b = 0, total = 0;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static long int_digits32_lc(size_t na, size_t nb) { return (long)((na + 1) / 2 + (nb + 1) / 2 - 1); }

static void int_layout_sizes(size_t na, size_t nb, IntLayout* L) {
  L->lc = L->d32 ? int_digits32_lc(na, nb) : (long)(na + nb - 1);
  L->x_b = align256((size_t)L->lc * (L->d32 ? 16 : 8));
  L->res_b = L->fused ? 0 : align256((size_t)L->lc * 4);
  L->wid_b = L->widen ? align256((na + nb) * 4) : 0;
  const size_t pw = L->fused ? 3 * align256(L->pw) : align256(L->pw);
  L->jobs_b = L->fused ? align256(3 * sizeof(ConvJob)) : 0;
  // the carries' state: one word per run of limbs (or of 32-bit words)
  const long units = L->d32 ? (long)((na + nb + 1) / 2) : (long)(na + nb);
  L->total = 3 * L->res_b + L->wid_b + pw + L->jobs_b + L->x_b + align256(carry_workspace_bytes(units));
}

// the plans the policy picks (plan choice may consult the cost model, so
// this runs at call time)
// The fused passes take the first radix 16, or 32 with at least 29 blocks
// kept; a plan of first radix 32 with fewer kept blocks runs as its twin of
// first radix 16 (the second column radix doubled, or the rows doubled when
// it is 32 already), so that the three primes still share their passes.
static Plan int3_twin(const Plan& P, long lc, int pidx) {
  if (P.kind != PLAN_FOURSTEP || P.logRA != 5 || int3_fused_ok(P)) return P;
  Plan T = P;
  T.logRA = 4;
  T.logRB = P.logRB + 1;
  if (T.logRB > 5) {
    T.logRB = 5;
    T.logC = P.logC + 1;
    T.lnt = std::min(10, plan_row_lnt(P) + 1);
  }
  T.ma = kept_blocks(lc, T.logL, 4);
  return plan_valid(T, lc, pidx) && int3_fused_ok(T) ? T : P;
}

// 32-bit digits: the three primes' plans at the digit product's length,
// usable when they are one plan with the fused three-prime passes
static bool int_layout_d32(size_t na, size_t nb, IntLayout* L) {
  const long dc = int_digits32_lc(na, nb);
  if (dc < 2) return false;
  for (int i = 0; i < 3; ++i) {
    const int pidx = prime_index(kIntPrimes[i]);
    L->plans[i] = int3_twin(choose_plan(dc, pidx), dc, pidx);
    if (!plan_valid(L->plans[i], dc, pidx)) return false;
  }
  if (!int3_fused_ok(L->plans[0]) || !same_plan(L->plans[0], L->plans[1]) || !same_plan(L->plans[0], L->plans[2]))
    return false;
  L->fused = true;
  L->d32 = true;
  L->widen = false;
  L->pw = plan_workspace_bytes(L->plans[0]);
  int_layout_sizes(na, nb, L);
  return true;
}

// digits: 0 (32-bit digits where their plans allow, else 16), 16 or 32
static pm_status int_mul_layout(size_t na, size_t nb, int digits, IntLayout* L) {
  const long lc = (long)(na + nb - 1);
  if (ceil_log2(lc) > 23) return PM_ETOOLARGE;
  if (digits != 0 && digits != 16 && digits != 32) return PM_EINVAL;
  if (digits != 16) {
    IntLayout D;
    if (int_layout_d32(na, nb, &D)) {
      *L = D;
      return PM_OK;
    }
    if (digits == 32) return PM_EUNSUPPORTED;
  }
  for (int i = 0; i < 3; ++i) {
    const int pidx = prime_index(kIntPrimes[i]);
    L->plans[i] = int3_twin(choose_plan(lc, pidx), lc, pidx);
    if (!plan_valid(L->plans[i], lc, pidx)) return PM_ETOOLARGE;
    if (L->plans[i].kind != PLAN_FOURSTEP) L->widen = true;
    L->pw = std::max(L->pw, plan_workspace_bytes(L->plans[i]));
  }
  // the three primes are below 2^30 (one value range), so equal plans can share launches
  L->fused = int3_fused_ok(L->plans[0]) && same_plan(L->plans[0], L->plans[1]) && same_plan(L->plans[0], L->plans[2]);
  int_layout_sizes(na, nb, L);
  return PM_OK;
}

pm_status pm_int_mul_digits_workspace_query(size_t na, size_t nb, int digit_bits, size_t* bytes) {
  if (!bytes || na == 0 || nb == 0) return PM_EINVAL;
  if (digit_bits != 0 && digit_bits != 16 && digit_bits != 32) return PM_EINVAL;
  const long lc = (long)(na + nb - 1);
  if (ceil_log2(lc) > 23) return PM_ETOOLARGE;
  // on the host alone: under the default policy (or with every prime's plan
  // put by the caller) the plans the call will use; otherwise (the cost model
  // picks at call time) the most any candidate plan could need, in the
  // layout that needs more
  bool known = current_policy() == PM_POLICY_DEFAULT;
  if (!known) {
    known = true;
    for (int i = 0; i < 3; ++i) known = known && plan_pinned(lc, kIntPrimes[i]);
  }
  if (known && digit_bits != 16) {
    const long dc = int_digits32_lc(na, nb);
    for (int i = 0; i < 3; ++i) known = known && (current_policy() == PM_POLICY_DEFAULT || plan_pinned(dc, kIntPrimes[i]));
  }
  IntLayout L;
  if (known) {
    const pm_status st = int_mul_layout(na, nb, digit_bits, &L);
    if (st) return st;
    *bytes = L.total;
    return PM_OK;
  }
  size_t worst = 0;
  if (digit_bits != 32) {
    size_t pw = 0;
    for (int i = 0; i < 3; ++i) pw = std::max(pw, product_workspace_bound(lc, prime_index(kIntPrimes[i])));
    for (int fused = 0; fused < 2; ++fused) {
      IntLayout W;
      W.pw = pw;
      W.widen = !fused;
      W.fused = fused != 0;
      int_layout_sizes(na, nb, &W);
      worst = std::max(worst, W.total);
    }
  }
  if (digit_bits != 16) {
    const long dc = int_digits32_lc(na, nb);
    if (dc >= 2) {
      IntLayout W;
      for (int i = 0; i < 3; ++i) W.pw = std::max(W.pw, product_workspace_bound(dc, prime_index(kIntPrimes[i])));
      W.fused = true;
      W.d32 = true;
      int_layout_sizes(na, nb, &W);
      worst = std::max(worst, W.total);
    }
  }
  *bytes = worst;
  return PM_OK;
}

pm_status pm_int_mul_workspace_query(size_t na, size_t nb, size_t* bytes) {
  return pm_int_mul_digits_workspace_query(na, nb, 0, bytes);
}

pm_status pm_int_mul_digits(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, int digit_bits,
                            uint16_t* out, void* stream) {
  if (!a || !b || !out || na == 0 || nb == 0) return PM_EINVAL;
  if (digit_bits != 0 && digit_bits != 16 && digit_bits != 32) return PM_EINVAL;
  const long lc0 = (long)(na + nb - 1);
  if (ceil_log2(lc0) > 23) return PM_ETOOLARGE;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  hipStream_t s = (hipStream_t)stream;
  const long nl = (long)(na + nb);
  IntLayout LY;
  st = int_mul_layout(na, nb, digit_bits, &LY);
  if (st) return st;
  const long lc = LY.lc;
  void* wsp = nullptr;
  st = stream_workspace(c, s, LY.total, &wsp);
  if (st) return st;
  char* base = (char*)wsp;
  u32* res[3] = {(u32*)base, (u32*)(base + LY.res_b), (u32*)(base + 2 * LY.res_b)};
  u32* wa = (u32*)(base + 3 * LY.res_b);
  u32* wb = wa + na;
  char* pws = base + 3 * LY.res_b + LY.wid_b;
  const size_t pw1 = align256(LY.pw);
  ConvJob* djobs = (ConvJob*)(pws + (LY.fused ? 3 * pw1 : pw1));
  u64* X = (u64*)((char*)djobs + LY.jobs_b);
  void* cws = (char*)X + LY.x_b;
  if (LY.fused) {
    // each pass once over the three primes; the residues never leave the inverse column pass
    const Plan& P = LY.plans[0];
    ConvJob J[3];
    for (int i = 0; i < 3; ++i) {
      u32* Ta = (u32*)(pws + i * pw1);
      st = make_job(c, P, prime_index(kIntPrimes[i]), a, (long)na, b, (long)nb, nullptr, lc, Ta, Ta + plan_nprime(P),
                    &J[i], 0);
      if (st) return st;
    }
    JobRef jr;
    jr.one = J[0];
    jr.many = djobs;
    hipError_t e = launch_col_fwd_int3(P, J, djobs, LY.d32, s);
    if (e == hipSuccess) e = launch_row_conv(P, true, J[0].rows, jr, 3, s);
    if (e == hipSuccess) e = launch_col_inv_crt3(P, djobs, X, LY.d32, s);
    if (e == hipSuccess) e = LY.d32 ? launch_carry32(X, lc, nl, cws, out, s) : launch_carry(X, lc, nl, cws, out, s);
    return dev_status(e);
  }
  if (LY.widen) {
    hipError_t e = launch_widen(a, (long)na, wa, s);
    if (e == hipSuccess) e = launch_widen(b, (long)nb, wb, s);
    if (e != hipSuccess) return PM_EDEVICE;
  }
  for (int i = 0; i < 3; ++i) {
    const int pidx = prime_index(kIntPrimes[i]);
    if (LY.plans[i].kind == PLAN_FOURSTEP)
      st = run_product(c, LY.plans[i], a, (long)na, b, (long)nb, 1, res[i], lc, pidx, pws, s);
    else
      st = run_product(c, LY.plans[i], wa, (long)na, wb, (long)nb, 0, res[i], lc, pidx, pws, s);
    if (st) return st;
  }
  hipError_t e = launch_crt_x(res[0], res[1], res[2], lc, X, s);
  if (e == hipSuccess) e = launch_carry(X, lc, nl, cws, out, s);
  return dev_status(e);
}

pm_status pm_int_mul(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint16_t* out, void* stream) {
  return pm_int_mul_digits(a, na, b, nb, 0, out, stream);
}

}  // extern "C"
