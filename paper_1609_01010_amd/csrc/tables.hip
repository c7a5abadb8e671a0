// Twiddle-table generation (GPU kernels) and the per-device context.
//
// The transforms need principal roots of unity of the coefficient ring, the
// w_N = g^((p-1)/N) that the convolution theorem evaluates at (section 3,
// eq. 10), and their powers, each stored with its Shoup companion
// floor(w * 2^32 / p).
#include <cstdio>
#include <cstdlib>

#include <vector>

#include "internal.h"

namespace pm {

static const PrimeInfo kPrimes[kNumPrimes] = {
    {998244353u, 3u, 23, 0u, true},
    {2013265921u, 31u, 27, 0u, false},
    {469762049u, 3u, 26, 0u, true},
    {167772161u, 3u, 25, 0u, true},
};

static u32 neg_inv32(u32 p) {
  // Newton iteration for p^-1 mod 2^32 (p odd), then negate
  u32 x = p;  // correct to 3 bits
  for (int i = 0; i < 5; ++i) x *= 2u - p * x;
  return 0u - x;
}

static PrimeInfo g_primes[kNumPrimes];
static std::once_flag g_primes_once;

static void init_primes() {
  for (int i = 0; i < kNumPrimes; ++i) {
    g_primes[i] = kPrimes[i];
    g_primes[i].ninv = neg_inv32(kPrimes[i].p);
  }
}

int prime_index(u32 p) {
  for (int i = 0; i < kNumPrimes; ++i)
    if (kPrimes[i].p == p) return i;
  return -1;
}

const PrimeInfo& prime_info(int pidx) {
  std::call_once(g_primes_once, init_primes);
  return g_primes[pidx];
}

u32 h_mulmod(u32 a, u32 b, u32 p) { return (u32)(((u64)a * b) % p); }
u32 h_powmod(u32 b, u64 e, u32 p) {
  u64 r = 1 % p, x = b % p;
  while (e) {
    if (e & 1) r = r * x % p;
    x = x * x % p;
    e >>= 1;
  }
  return (u32)r;
}
u32 h_inv(u32 a, u32 p) { return h_powmod(a, p - 2, p); }
uint2 h_shoup(u32 w, u32 p) { return make_uint2(w, (u32)(((u64)w << 32) / p)); }

// ---------------------------------------------------------------------------
// kernels

__device__ __forceinline__ u32 d_mulmod(u32 a, u32 b, u32 p) { return (u32)(((u64)a * b) % p); }
__device__ u32 d_powmod(u32 b, u32 e, u32 p) {
  u32 r = 1, x = b;
  while (e) {
    if (e & 1) r = d_mulmod(r, x, p);
    x = d_mulmod(x, x, p);
    e >>= 1;
  }
  return r;
}
__device__ __forceinline__ uint2 d_shoup(u32 w, u32 p) { return make_uint2(w, (u32)(((u64)w << 32) / p)); }

// Pyramids: pf[2^s + x] = w_{2^s}^x, pi[2^s + x] = w_{2^s}^-x (s <= 15),
// ph[2^s + x] = w_{2^s}^-x / 2 (s <= 5), iv[k] = 2^-k.
__global__ void k_fill_pyramids(uint2* base, u32 p, u32 g) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  uint2* pf = base;
  uint2* pi = base + kPyrSize;
  uint2* ph = pi + kPyrSize;
  uint2* iv = ph + kHalfSize;
  if (idx >= 1 && idx < kPyrSize) {
    const int s = 31 - __clz(idx);
    const u32 x = (u32)idx - (1u << s);
    const u32 w = d_powmod(g, (p - 1) >> s, p);  // primitive 2^s-th root
    const u32 wf = d_powmod(w, x, p);
    const u32 wi = d_powmod(w, ((1u << s) - x) & ((1u << s) - 1), p);
    pf[idx] = d_shoup(wf, p);
    pi[idx] = d_shoup(wi, p);
    if (idx < kHalfSize) ph[idx] = d_shoup(d_mulmod(wi, (p + 1) / 2, p), p);
  }
  if (idx == 0) {
    pf[0] = pi[0] = make_uint2(0, 0);
    ph[0] = make_uint2(0, 0);
  }
  if (idx < kInvPow) iv[idx] = d_shoup(d_powmod((p + 1) / 2, (u32)idx, p), p);
}

// Round tables for radix Q = 2^lq: level B = 2^s (Q <= B <= 2^15),
// out[B + j Q + t] = w_B^{sign j rev_lq(t)}, j < B/Q, t < Q.
__global__ void k_fill_round_table(uint2* out, u32 p, u32 g, int lq, int inverse) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int Q = 1 << lq;
  if (idx < Q || idx >= kPyrSize) {
    if (idx < Q) out[idx] = make_uint2(0, 0);
    return;
  }
  const int s = 31 - __clz(idx);
  const u32 o = (u32)idx - (1u << s);
  const u32 j = o >> lq, t = o & (Q - 1);
  const u32 rt = __brev(t) >> (32 - lq);
  const u32 w = d_powmod(g, (p - 1) >> s, p);
  u32 e = (j * rt) & ((1u << s) - 1);
  if (inverse) e = ((1u << s) - e) & ((1u << s) - 1);
  out[idx] = d_shoup(d_powmod(w, e, p), p);
}

// Row-pass twiddle factors.  With kf = kmul k1 + kadd (k1 for the cyclic
// transform, 2 k1 + 1 for the twisted one of the nega-circular product):
//   out[k1 * ept + e] = mult * base^((nt e kf) mod ord)     (k_row_factors)
//   out[k1 * nt + tid] = base^(tid kf)                       (k_row_pows)
// ord is the order of base (a power of two).
__global__ void k_row_factors(uint2* out, int R, int ept, int nt, u32 ord_mask, u32 p, u32 base, u32 mult, u32 kmul,
                              u32 kadd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * ept) return;
  const u64 k1 = (u64)(i / ept), e = (u64)(i % ept);
  const u32 ex = (u32)(((u64)nt * e * (kmul * k1 + kadd)) & ord_mask);
  out[i] = d_shoup(d_mulmod(mult, d_powmod(base, ex, p), p), p);
}

__global__ void k_row_pows(uint2* out, int R, int nt, u32 ord_mask, u32 p, u32 base, u32 kmul, u32 kadd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * nt) return;
  const u64 k1 = (u64)(i / nt), tid = (u64)(i % nt);
  out[i] = d_shoup(d_powmod(base, (u32)((tid * (kmul * k1 + kadd)) & ord_mask), p), p);
}

// out[i] = base^i as Shoup pairs, i < n
__global__ void k_pows(uint2* out, int n, u32 p, u32 base) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = d_shoup(d_powmod(base, (u32)i, p), p);
}

// ---------------------------------------------------------------------------
// per-device context

static std::mutex g_ctx_mu;
static std::map<int, DevCtx*> g_ctx;

DevCtx* ctx_lookup() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  return it == g_ctx.end() ? nullptr : it->second;
}

DevCtx* ctx_current(pm_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *st = PM_EDEVICE;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) {
    *st = PM_OK;
    return it->second;
  }
  DevCtx* c = new DevCtx();
  c->dev = dev;
  if (hipMalloc(&c->errflag, sizeof(int)) != hipSuccess) {
    delete c;
    *st = PM_ENOMEM;
    return nullptr;
  }
  if (hipMemset(c->errflag, 0, sizeof(int)) != hipSuccess) {
    *st = PM_EDEVICE;
    return nullptr;
  }
  *st = mlp_infer_init(&c->infer);
  if (*st) return nullptr;
  g_ctx[dev] = c;
  *st = PM_OK;
  return c;
}

// Completion matrices of truncated inverses (the kx table): the inverse
// transform of size Q = 2^q maps bit-reversed outputs x to Q z with
// G[j][t] = w_Q^{-j rev_q(t)}.  When z_j = 0 for j >= M = Q - d, the rows
// j >= M give G_m x_miss + G_k x_known = 0, so K = -G_m^-1 G_k (G_m: the
// columns t >= M, invertible as a Vandermonde matrix at distinct points,
// scaled); Gauss-Jordan elimination mod p.
static void fill_completion(const PrimeInfo& P, std::vector<uint2>& out) {
  out.assign(kFillSize, make_uint2(0, 0));
  const u32 p = P.p;
  for (int lq = kFillMinLog; lq <= kFillMaxLog; ++lq) {
    const int Q = 1 << lq;
    const u32 wi = h_inv(h_powmod(P.g, (p - 1) / (u32)Q, p), p);
    auto rev = [lq](int t) {
      int r = 0;
      for (int b = 0; b < lq; ++b) r |= ((t >> b) & 1) << (lq - 1 - b);
      return r;
    };
    for (int d = 1; d <= kFillMax; ++d) {
      const int M = Q - d;
      // augmented rows [G_m | -G_k] for j = M .. Q-1
      std::vector<std::vector<u32>> a(d, std::vector<u32>(Q));
      for (int r = 0; r < d; ++r) {
        const int j = M + r;
        for (int t = 0; t < Q; ++t) {
          const u32 gv = h_powmod(wi, (u64)j * (u64)rev(t), p);
          if (t >= M)
            a[r][t - M] = gv;
          else
            a[r][d + t] = gv ? p - gv : 0u;
        }
      }
      for (int col = 0; col < d; ++col) {
        int piv = col;
        while (piv < d && a[piv][col] == 0) ++piv;
        if (piv == d) continue;  // not reached: G_m is invertible
        std::swap(a[piv], a[col]);
        const u32 inv = h_inv(a[col][col], p);
        for (auto& v : a[col]) v = h_mulmod(v, inv, p);
        for (int r = 0; r < d; ++r) {
          if (r == col || a[r][col] == 0) continue;
          const u32 f = a[r][col];
          for (int k = 0; k < Q; ++k) a[r][k] = (u32)((a[r][k] + (u64)(p - h_mulmod(f, a[col][k], p))) % p);
        }
      }
      uint2* K = out.data() + fill_offset(lq, d);
      for (int r = 0; r < d; ++r)
        for (int k = 0; k < M; ++k) K[r * M + k] = h_shoup(a[r][d + k], p);
    }
  }
}

pm_status ensure_prime_tables(DevCtx* c, int pidx) {
  if (c->prime_mem[pidx]) return PM_OK;
  const PrimeInfo& P = prime_info(pidx);
  // pf, pi, ph, iv, then the round tables (Q = 2 .. 32; both directions),
  // then the completion matrices
  const size_t head = 2 * (size_t)kPyrSize + kHalfSize + kInvPow;
  const size_t head_al = (head + 63) & ~(size_t)63;
  const size_t kx_at = head_al + 2 * kRoundTables * (size_t)kPyrSize;
  const size_t n = kx_at + kFillSize;
  std::vector<uint2> kx;
  fill_completion(P, kx);
  uint2* mem = nullptr;
  if (hipMalloc(&mem, n * sizeof(uint2)) != hipSuccess) return PM_ENOMEM;
  k_fill_pyramids<<<kPyrSize / 256, 256>>>(mem, P.p, P.g);
  for (int q = 0; q < kRoundTables; ++q) {
    k_fill_round_table<<<kPyrSize / 256, 256>>>(mem + head_al + (2 * q) * kPyrSize, P.p, P.g, q + 1, 0);
    k_fill_round_table<<<kPyrSize / 256, 256>>>(mem + head_al + (2 * q + 1) * kPyrSize, P.p, P.g, q + 1, 1);
  }
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(mem + kx_at, kx.data(), kFillSize * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(mem);
    return PM_EDEVICE;
  }
  c->prime_mem[pidx] = mem;
  c->tabs[pidx].pf = mem;
  c->tabs[pidx].pi = mem + kPyrSize;
  c->tabs[pidx].ph = mem + 2 * kPyrSize;
  c->tabs[pidx].iv = mem + 2 * kPyrSize + kHalfSize;
  for (int q = 0; q < kRoundTables; ++q) {
    c->tabs[pidx].rf[q] = mem + head_al + (2 * q) * kPyrSize;
    c->tabs[pidx].ri[q] = mem + head_al + (2 * q + 1) * kPyrSize;
  }
  c->tabs[pidx].kx = mem + kx_at;
  return PM_OK;
}

size_t row_tables_bytes(int logL, int logC, int lnt) {
  const size_t R = (size_t)1 << (logL - logC), nt = (size_t)1 << lnt, ept = (size_t)1 << (logC - lnt);
  return 2 * (R * nt + R * ept) * sizeof(uint2);
}

pm_status fill_row_tables(int pidx, int logL, int logC, int lnt, u32 scale, int twist, uint2* mem, hipStream_t s,
                          RowTables* out) {
  const PrimeInfo& P = prime_info(pidx);
  const int R = 1 << (logL - logC), nt = 1 << lnt, ept = 1 << (logC - lnt);
  const int ng = R * nt, nf = R * ept;
  if (twist && logL + 1 > P.two_adic) return PM_ETOOLARGE;
  // cyclic: w_L^(j2 k1); twisted: psi^(j2 (2 k1 + 1)) with psi^2 = w_L
  const int lord = twist ? logL + 1 : logL;
  const u32 w = h_powmod(P.g, (P.p - 1) >> lord, P.p);
  const u32 wi = h_inv(w, P.p);
  const u32 mask = (u32)((1ull << lord) - 1);
  const u32 kmul = twist ? 2 : 1, kadd = twist ? 1 : 0;
  uint2* gf = mem;
  uint2* gi = gf + ng;
  uint2* ff = gi + ng;
  uint2* fi = ff + nf;
  k_row_pows<<<(ng + 255) / 256, 256, 0, s>>>(gf, R, nt, mask, P.p, w, kmul, kadd);
  k_row_pows<<<(ng + 255) / 256, 256, 0, s>>>(gi, R, nt, mask, P.p, wi, kmul, kadd);
  k_row_factors<<<(nf + 255) / 256, 256, 0, s>>>(ff, R, ept, nt, mask, P.p, w, 1, kmul, kadd);
  k_row_factors<<<(nf + 255) / 256, 256, 0, s>>>(fi, R, ept, nt, mask, P.p, wi, scale, kmul, kadd);
  if (hipGetLastError() != hipSuccess) return PM_EDEVICE;
  out->gf = gf;
  out->gi = gi;
  out->ff = ff;
  out->fi = fi;
  return PM_OK;
}

pm_status get_row_tables(DevCtx* c, int pidx, int logL, int logC, int lnt, u32 scale, int twist, RowTables* out) {
  const RowKey key{pidx, logL, logC, lnt, scale, twist};
  auto it = c->rowtw.find(key);
  if (it != c->rowtw.end()) {
    *out = it->second.second;
    return PM_OK;
  }
  if (twist && logL + 1 > prime_info(pidx).two_adic) return PM_ETOOLARGE;
  uint2* mem = nullptr;
  if (hipMalloc(&mem, row_tables_bytes(logL, logC, lnt)) != hipSuccess) return PM_ENOMEM;
  RowTables W;
  pm_status st = fill_row_tables(pidx, logL, logC, lnt, scale, twist, mem, 0, &W);
  if (st == PM_OK && hipDeviceSynchronize() != hipSuccess) st = PM_EDEVICE;
  if (st) {
    hipFree(mem);
    return st;
  }
  c->rowtw[key] = std::make_pair(mem, W);
  *out = W;
  return PM_OK;
}

pm_status get_twist_tables(DevCtx* c, int pidx, int logL, int log_stride, const uint2** fwd, const uint2** inv) {
  const RowKey key{pidx, logL, log_stride, -1, 0u, 1};
  auto it = c->rowtw.find(key);
  if (it == c->rowtw.end()) {
    const PrimeInfo& P = prime_info(pidx);
    if (logL + 1 > P.two_adic) return PM_ETOOLARGE;
    const int n = 1 << (logL - log_stride);
    uint2* mem = nullptr;
    if (hipMalloc(&mem, 2 * (size_t)n * sizeof(uint2)) != hipSuccess) return PM_ENOMEM;
    // psi, a primitive 2L-th root of unity (psi^L = -1), raised to the stride
    const u32 psi = h_powmod(P.g, (P.p - 1) >> (logL + 1), P.p);
    const u32 base = h_powmod(psi, 1u << log_stride, P.p);
    k_pows<<<(n + 255) / 256, 256>>>(mem, n, P.p, base);
    k_pows<<<(n + 255) / 256, 256>>>(mem + n, n, P.p, h_inv(base, P.p));
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      hipFree(mem);
      return PM_EDEVICE;
    }
    RowTables W{};
    W.gf = mem;
    W.gi = mem + n;
    it = c->rowtw.emplace(key, std::make_pair(mem, W)).first;
  }
  *fwd = it->second.second.gf;
  *inv = it->second.second.gi;
  return PM_OK;
}

void* stream_workspace_current(DevCtx* c, hipStream_t s) {
  auto u = c->user_ws.find(s);
  if (u != c->user_ws.end()) return u->second.first;
  auto it = c->ws.find(s);
  return it != c->ws.end() ? it->second.first : nullptr;
}

pm_status stream_workspace(DevCtx* c, hipStream_t s, size_t bytes, void** out) {
  auto u = c->user_ws.find(s);
  if (u != c->user_ws.end()) {
    if (u->second.second < bytes) return PM_ENOMEM;
    *out = u->second.first;
    return PM_OK;
  }
  auto& w = c->ws[s];
  if (w.second < bytes) {
    if (w.first) {
      // work already queued on s may still use the old buffer
      if (hipStreamSynchronize(s) != hipSuccess) return PM_EDEVICE;
      hipFree(w.first);
      w.first = nullptr;
      w.second = 0;
    }
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (hipMalloc(&w.first, want) != hipSuccess) return PM_ENOMEM;
    w.second = want;
  }
  *out = w.first;
  return PM_OK;
}

}  // namespace pm
