/*
 * polymul.h - C ABI of the MI355X (gfx950) modular polynomial multiplication
 * library: products over Z/pZ by number-theoretic transforms, following
 * L. Meng, "Automatic Library Generation for Modular Polynomial Multiplication".
 *
 * General conventions (apply to every call unless stated otherwise):
 *  - Coefficient arrays are little-endian in the degree: element i is the
 *    coefficient of x^i (Def. 1).  Elements are uint32 in canonical form
 *    [0, p); a value >= p is an error, detected on the device and reported
 *    as PM_ENOTREDUCED by pm_stream_check (it is never reduced silently).
 *  - All data pointers are DEVICE pointers on the current HIP device, owned by
 *    the caller (for instance torch tensors).  The library never frees them.
 *    Distinct arrays must not overlap.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it and the call returns after host-side validation;
 *    results are valid once the stream has reached that point.
 *  - p must be one of 998244353 (119*2^23+1, root 3), 2013265921 (15*2^27+1,
 *    root 31), 469762049 (7*2^26+1, root 3), 167772161 (5*2^25+1, root 3);
 *    other values give PM_EUNSUPPORTED.  A transform length L must divide
 *    p - 1 (L <= 2^23, 2^27, 2^26, 2^25 respectively, and L <= 2^24 overall);
 *    larger lengths give PM_ETOOLARGE.
 *  - A zero length or a NULL pointer gives PM_EINVAL.  Errors detected on the
 *    host leave the outputs untouched and enqueue nothing.
 *  - The library owns its twiddle tables, plan cache and workspace (allocated
 *    lazily per device with hipMalloc, freed at process exit).  Calls from
 *    several host threads are serialised per device.
 */
#ifndef POLYMUL_H
#define POLYMUL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PM_OK = 0,
  PM_EINVAL = 1,        /* bad argument: NULL pointer, zero length, bad size */
  PM_EUNSUPPORTED = 2,  /* modulus not among the four supported primes */
  PM_ETOOLARGE = 3,     /* transform length exceeds what p supports */
  PM_ENOTREDUCED = 4,   /* an input coefficient was >= p (reported late) */
  PM_ENOMEM = 5,        /* device allocation failed */
  PM_EDEVICE = 6        /* a HIP call or kernel launch failed */
} pm_status;

/* Text for a status code (static storage). */
const char* pm_status_str(pm_status s);

/* Initialise the library on the current device (optional: every call does it
 * on first use).  Builds the twiddle tables of all four primes.  The first
 * pm_init of a process also applies pm_config_from_env(); if that fails, this
 * and every later pm_init return its status. */
pm_status pm_init(void);

/*
 * Polynomial product (Def. 2, eq. 2; the linear convolution of Def. 3):
 *   c_k = sum_{i+j=k} a_i b_j mod p,   0 <= k <= len_a + len_b - 2.
 * a: len_a coefficients, b: len_b coefficients, c: len_a + len_b - 1 outputs.
 * Computed by the convolution theorem (Theorem 1, eq. 10): forward transforms
 * of both operands, n pointwise products, one inverse transform with scaling.
 * The transform is the padded power-of-two modular DFT (eq. 12) when
 * len_a + len_b - 1 is a power of two, otherwise a relaxed truncated Fourier
 * transform (TFT/ITFT, eq. 14) that computes n' >= len_a + len_b - 1 values,
 * n' a multiple of the plan's granularity, without padding to the next power
 * of two.  Products with fewer than 64 outputs use the defining sum directly.
 * Requires the transform length L (next power of two >= len_a + len_b - 1)
 * to be supported by p.  c must not overlap a or b.
 */
pm_status pm_poly_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p, uint32_t* c,
                      void* stream);

/*
 * pm_poly_mul for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same product as pm_poly_mul, computed by the same kernels, but every
 * intermediate (the four-step workspace and the row-pass factor tables of the
 * plan) lives in a static device array of 22 MiB that each device holds from
 * the library's load until the process ends; the call allocates nothing and
 * never waits for the device.
 *  - pm_init() must have run on the current device first (it finds the
 *    array's address there); otherwise PM_EINVAL.
 *  - The plan is the cached plan of the length (pm_plan_cache_put), else the
 *    default plan (also in place of a cached general-radix plan, kind 3);
 *    the cost model and the tuner are not consulted.
 *  - Products whose plan needs more than the array (a relaxed transform
 *    length n' above 2^21, i.e. len_a + len_b - 1 > 2^21 for the default
 *    plans) give PM_ETOOLARGE and launch nothing.
 *  - Every call on a device shares that device's array, which keeps the last
 *    call's contents (nothing in it needs to start at zero): calls on
 *    different streams of one device that overlap in time race on it, so
 *    order them (one stream, or events).
 * Other arguments and errors as pm_poly_mul.
 */
pm_status pm_poly_mul_noalloc(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                              uint32_t* c, void* stream);

/*
 * Products in the quotient rings of the factorisation of eq. 13:
 *   pm_cyclic_mul:     c = a b mod (x^n - 1), the circular convolution
 *                      (Def. 4, eq. 5): c_i = sum_{j+k = i mod n} a_j b_k;
 *   pm_negacyclic_mul: c = a b mod (x^n + 1), the nega-circular one:
 *                      c_i = sum_{j+k = i} a_j b_k - sum_{j+k = i+n} a_j b_k.
 * n is a power of two; len_a, len_b <= n (missing coefficients are zero);
 * c receives n outputs, canonical.  The circular product is one length-n
 * transform per operand, the pointwise product and one inverse (the
 * convolution theorem without padding, diagram 9); the nega-circular one is
 * the same on inputs twisted by psi^j (psi a primitive 2n-th root of unity,
 * psi^n = -1) with the output untwisted by psi^-j; the twists are folded into
 * the passes that read and write HBM and into the four-step row factors.
 * Requires n (cyclic) or 2n (nega-circular) to divide p - 1 and n <= 2^24;
 * n <= 64 uses the defining sums.  Errors as pm_poly_mul.
 */
pm_status pm_cyclic_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, size_t n, uint32_t p,
                        uint32_t* c, void* stream);
pm_status pm_negacyclic_mul(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, size_t n, uint32_t p,
                            uint32_t* c, void* stream);

/*
 * The product a * b mod p (as pm_poly_mul) through a circular convolution of
 * length N = q 2^k >= len_a + len_b - 1, q odd (general radix: section 1,
 * the smoothing of the power-of-two staircase by transforms of other
 * lengths): the prime-factor split of the length-N convolution into q
 * circular products of length 2^k by a length-q transform, and back.  q in
 * {3, 5, 7, 15, 17} dividing p - 1 (see pm_ntt), else PM_EUNSUPPORTED;
 * 2^k <= 2^24 and within p's 2-adic order, else PM_ETOOLARGE.  The q rows of
 * each operand and of the result live in the stream's workspace (3 N words).
 * Other errors as pm_poly_mul.
 */
pm_status pm_poly_mul_mixed(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p, uint32_t q,
                            uint32_t* c, void* stream);

/*
 * Dense multivariate product (section 1: multivariate products reduce to
 * univariate ones), here by Kronecker substitution: one univariate
 * product (pm_poly_mul) of the operands packed with the strides of the
 * product's box.  a is row-major over the box dims_a[0] x .. x
 * dims_a[nvars-1] (dims_a[i] = 1 + the degree of a in variable i, the last
 * variable fastest); likewise b.  c receives the product row-major over
 * dims_a[i] + dims_b[i] - 1.  dims_a, dims_b: HOST arrays; 1 <= nvars <= 8.
 * The packed operands live in the stream's workspace.  Requires the product's
 * number of coefficients to be a supported transform length (as pm_poly_mul).
 */
pm_status pm_poly_mul_multi(const uint32_t* a, const size_t* dims_a, const uint32_t* b, const size_t* dims_b,
                            int nvars, uint32_t p, uint32_t* c, void* stream);

/* One problem of a batch; all pointers are device pointers. */
typedef struct {
  const uint32_t* a;
  size_t len_a;
  const uint32_t* b;
  size_t len_b;
  uint32_t p;
  uint32_t* c; /* len_a + len_b - 1 outputs */
} pm_problem;

/*
 * Batch of independent products (each as pm_poly_mul), of uneven lengths and
 * mixed primes.  `probs` is a HOST array of `count` <= 65535 problems.  The
 * products are grouped into classes of equal plan (those of at most 64
 * outputs, computed by their defining sums, form one class, and so do, per
 * value range of the prime, the one-work-group products of 2^6 .. 2^11
 * points with first radix 8); each class runs
 * one launch per pass over all its products, and the classes are captured
 * into one hipGraph, cached by the batch's class signature.  A call whose problems
 * have the same lengths and primes, in order, as the previous call on the
 * stream only patches the pointers into the previous job descriptors and
 * relaunches.  Under PM_POLICY_LEARNED the plans come from the cost model in
 * the batch context, one plan family per transform length and prime; the
 * first call of a batch shape also runs the batch with the default plans,
 * waits for the device (the call is synchronous, and must not be made while
 * the stream is being captured), and keeps the faster plans for that shape.
 * On a host-side error no problem is computed.  Output arrays must be
 * pairwise disjoint.
 */
pm_status pm_poly_mul_batch(const pm_problem* probs, size_t count, void* stream);

/*
 * Workspace.  Products, transforms and batches keep their intermediate
 * arrays (the four-step passes' n' words per operand, the integer product's
 * residues and carry state) in one workspace per stream, which the library
 * allocates with hipMalloc on first use and grows as needed (growing waits
 * for the stream).  Callers that manage device memory themselves supply it:
 *
 *   pm_workspace_query:        bytes pm_poly_mul(len_a, len_b, p) needs: under
 *                              the default policy, for the cached or default
 *                              plan (0 for one-work-group and defining-sum
 *                              plans); under the learned and exhaustive
 *                              policies, whose plan is picked at call time,
 *                              the most any candidate plan needs.
 *   pm_batch_workspace_query:  bytes pm_poly_mul_batch needs for these
 *                              problems (host array).
 *   pm_int_mul_workspace_query: bytes pm_int_mul(na, nb) needs;
 *                              pm_int_mul_digits_workspace_query: bytes
 *                              pm_int_mul_digits(na, nb, digit_bits) needs.
 *   pm_set_workspace:          use the caller's device memory [ptr, ptr +
 *                              bytes) as the workspace of `stream` on the
 *                              current device from now on; a call that needs
 *                              more returns PM_ENOMEM and launches nothing.
 *                              ptr = NULL returns the stream to the library's
 *                              own workspace.  The caller keeps the memory
 *                              alive, and does not touch it, while work
 *                              queued on the stream may use it.  Twiddle
 *                              tables are still allocated by the library,
 *                              once per device and prime.
 * The queries need no device and validate their arguments as the calls do.
 */
pm_status pm_workspace_query(size_t len_a, size_t len_b, uint32_t p, size_t* bytes);
pm_status pm_batch_workspace_query(const pm_problem* probs, size_t count, size_t* bytes);
pm_status pm_int_mul_workspace_query(size_t na, size_t nb, size_t* bytes);
pm_status pm_int_mul_digits_workspace_query(size_t na, size_t nb, int digit_bits, size_t* bytes);
pm_status pm_set_workspace(void* stream, void* ptr, size_t bytes);

/*
 * Integer product by the three-primes algorithm (section 1): A and B are
 * little-endian integers of na and nb 16-bit limbs (A = sum a_i 2^{16 i}).
 * Their digit sequences are multiplied as polynomials modulo 469762049,
 * 998244353 and 167772161, the three residues of every coefficient are
 * combined by the Chinese remainder theorem into the exact sum (< 2^54 for
 * 16-bit digits, < 2^85 for 32-bit ones; p1 p2 p3 is about 2^86.02), and
 * carries are propagated.  c receives exactly na + nb limbs of A*B (the top
 * limb may be 0).  Requires na + nb - 1 <= 2^23.
 * Digits: pm_int_mul takes 32-bit digits (digit j = a_{2j} + 2^16 a_{2j+1},
 * so the transforms have ceil(na/2) + ceil(nb/2) - 1 points, half as many)
 * when the three primes' plans at that length are one plan with the fused
 * passes described below, else the 16-bit limbs themselves.
 * pm_int_mul_digits chooses with digit_bits = 0 in the same way, and forces
 * 16 or 32 (32 returns PM_EUNSUPPORTED where the plans do not allow it);
 * another value is PM_EINVAL.  The digits change the cost, never the result.
 * Plans: for each prime, the plan of the transform's output length (na +
 * nb - 1, or the digit product's length above) in the product-alone
 * context: the cached one (pm_plan_cache_put, or the tuner's
 * pick after pm_tune), else under PM_POLICY_LEARNED the cost model's pick,
 * else the default plan.  The call never times candidates itself: under
 * PM_POLICY_EXHAUSTIVE an untuned length takes the default plan (tune it
 * for the three primes first).  When the three plans are one four-step plan
 * of first radix 16, or 32 with at least 29 of its blocks kept, each pass
 * runs once for the three primes and the CRT is taken inside the inverse
 * pass (a plan of first radix 32 with fewer kept blocks runs as its twin of
 * first radix 16 for this); otherwise each prime's product runs on its own
 * and the CRT reads the three residue arrays.
 */
pm_status pm_int_mul(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, uint16_t* c, void* stream);
pm_status pm_int_mul_digits(const uint16_t* a, size_t na, const uint16_t* b, size_t nb, int digit_bits, uint16_t* c,
                            void* stream);

/*
 * Length-n modular DFT (section 3: evaluation at w^0 .. w^{n-1}, with
 * w = g^((p-1)/n)), natural order in and out, 2 <= n.  n is a power of two,
 * or n = q 2^k with q in {3, 5, 7, 15, 17} (the general-size transforms of
 * the library generator that section 1 builds on): then q must divide p - 1
 * (3, 5, 15 for 2013265921; 7, 17 for 998244353; 7 for 469762049; 5 for
 * 167772161) and is split off by the prime-factor algorithm.  inverse != 0
 * computes the inverse transform including the factor n^-1.  x: n inputs;
 * y: n outputs (may equal x).  Errors: PM_EUNSUPPORTED for an odd part of n
 * that is not supported for p, PM_ETOOLARGE for 2^k beyond p's 2-adic order
 * or 2^24.
 */
pm_status pm_ntt(const uint32_t* x, uint32_t* y, size_t n, uint32_t p, int inverse, void* stream);

/*
 * Truncated Fourier transform TFT(L, z, n) (section 3, the TFT product):
 *   out_i = sum_{j<z} x_j w_L^{j rev_l(i)},  0 <= i < n,
 * with rev_l the bit reversal on l = log2 L bits (the first n values of the
 * length-L transform in bit-reversed order).  L a power of two, 1 <= z <= L,
 * 1 <= n <= L.  x: z inputs; out: n outputs.
 */
pm_status pm_tft(const uint32_t* x, size_t z, size_t L, size_t n, uint32_t p, uint32_t* out, void* stream);

/*
 * Inverse truncated Fourier transform ITFT(L, n, n): given the n values
 * v_i = u(w_L^{rev_l(i)}) of a polynomial u of degree < n, returns
 * (L u_0, ..., L u_{n-1}), the scaling the paper states for the ITFT.
 * v: n inputs; out: n outputs.  n must be a multiple of the granularity
 * pm_itft_granularity(L) (every n when L <= 32); otherwise PM_EINVAL.
 */
pm_status pm_itft(const uint32_t* v, size_t L, size_t n, uint32_t p, uint32_t* out, void* stream);

/* Granularity of the relaxed truncation for transform length L: the
 * multiple n' of the relaxed transforms is taken in steps of this size. */
size_t pm_itft_granularity(size_t L);

/*
 * Wait for `stream` and report errors detected on the device since the last
 * check on this device (PM_ENOTREDUCED), or PM_EDEVICE if the stream failed.
 * Clears the device error state.
 */
pm_status pm_stream_check(void* stream);

/* ---- plans, tuning and the learned cost model --------------------------- */

typedef enum { PM_POLICY_DEFAULT = 0, PM_POLICY_EXHAUSTIVE = 1, PM_POLICY_LEARNED = 2 } pm_policy;

/* Plan description (see pm_plan_for / pm_poly_mul_plan). */
typedef struct {
  int32_t kind;  /* 0: defining sum, 1: one work-group in LDS, 2: four-step,
                    3: general radix (as pm_poly_mul_mixed: q circular row
                    products of length 2^log_l; the other fields unused) */
  int32_t log_l; /* transform length L = 2^log_l */
  int32_t log_ra; /* first radix (the truncated one) */
  int32_t log_rb; /* second column radix of the four-step (0: none) */
  int32_t log_c;  /* row length of the four-step (LDS tile) */
  int32_t ma;     /* kept blocks of the first radix, 1 .. 2^log_ra */
  int32_t lq;     /* log radix of the LDS rounds */
  int32_t lnt;    /* log2 threads per row work-group of the four-step (0: default) */
  int32_t q;      /* kind 3: the odd factor (3 or 5) */
} pm_plan;

/* Select the policy used by pm_poly_mul / pm_poly_mul_batch to pick plans. */
pm_status pm_set_policy(pm_policy policy);
/* The policy in force (PM_POLICY_DEFAULT until one is set). */
pm_policy pm_get_policy(void);
/* Plan choice from the process environment (host only; needs no device):
 *   PM_PLAN_POLICY  "default", "exhaustive" or "learned": pm_set_policy;
 *   PM_TUNE_DB      path of a timing database: pm_tune_db_load (appends);
 *   PM_MLP_WEIGHTS  path of cost-model weights: pm_model_load.
 * Unset or empty variables change nothing.  Another policy name gives
 * PM_EINVAL before anything is applied; otherwise the database and the model
 * load first (their status is returned at the first failure, leaving the
 * rest unapplied) and the policy is set last.  May be called again to re-read
 * the environment. */
pm_status pm_config_from_env(void);

/* Timing contexts of the tuner, the database and the cost model.  A product
 * on its own is bound by its own parallelism (its plan should spread it over
 * the device); one of a batch shares the device with the others (its plan
 * should do the least work and traffic).  pm_poly_mul and the hooks choose
 * plans for PM_CTX_SINGLE, pm_poly_mul_batch for PM_CTX_BATCH; the plan cache
 * holds one entry per (length, prime, context). */
#define PM_CTX_SINGLE 0
#define PM_CTX_BATCH 1

/* The plan the current policy picks for an output length lc and prime p:
 * for a product on its own (pm_plan_for), or in a context.  In the batch
 * context under PM_POLICY_LEARNED, pm_poly_mul_batch plans a batch's new
 * lengths together (one plan family per transform length and prime) and
 * caches them; before that, a length gets the model's own pick. */
pm_status pm_plan_for(size_t lc, uint32_t p, pm_plan* plan);
pm_status pm_plan_for_ctx(size_t lc, uint32_t p, int context, pm_plan* plan);

/*
 * The plans the last pm_poly_mul_batch call on `stream` (current device)
 * used, problem by problem (kind 0 for the defining sums), into the HOST
 * array out of `count` entries; PM_EINVAL if no batch ran on the stream or
 * its size was not `count`.
 */
pm_status pm_batch_plans_used(void* stream, pm_plan* out, size_t count);

/* Product with an explicit plan (validated; PM_EINVAL if it does not fit). */
pm_status pm_poly_mul_plan(const uint32_t* a, size_t len_a, const uint32_t* b, size_t len_b, uint32_t p,
                           uint32_t* c, const pm_plan* plan, void* stream);

/* Number of candidate plans for (lc, p) and the i-th one (the tuner's space):
 * the power-of-two plans (kinds 0-2), then the general-radix plans (kind 3:
 * for each supported odd q dividing p - 1, the shortest q 2^k >= lc, where
 * it is shorter than the power of two).  Kind 3 runs for products alone:
 * the batch executor, the tuner's PM_CTX_BATCH and the cost model take the
 * power-of-two plans only. */
size_t pm_plan_candidates(size_t lc, uint32_t p, pm_plan* out, size_t max_out);

/* Record the plan to use for (lc, p) in the plan cache, for both contexts
 * (used by all policies before they choose); a general-radix plan (kind 3)
 * for products alone only. */
pm_status pm_plan_cache_put(size_t lc, uint32_t p, const pm_plan* plan);
void pm_plan_cache_clear(void);

/* ---- the autotuner (empirical search) -------------------------------------
 * The tuner times every candidate plan of an output length on the device
 * (hipEvents, median of `reps` runs after a warm-up, deterministic inputs)
 * and records (length, prime, plan, microseconds, context) in the in-memory
 * timing database; the fastest plan of each length goes to the plan cache of
 * that context.  This follows the paper's search over measured running times
 * (section 2.2, and the autotuned library of section 5).  In PM_CTX_SINGLE a
 * plan is timed on one product; in PM_CTX_BATCH on about 2^24 / L products
 * of the length at once (at most 4096: enough to fill the device whatever the
 * plan) (each pass one launch over all of them, as the batch
 * executor runs a class), and the time per product is recorded.  Products
 * alone also time the general-radix plans (kind 3).
 * Synchronous: returns after timing.  pm_tune is pm_tune_ctx(.., PM_CTX_SINGLE). */
pm_status pm_tune(const size_t* lcs, size_t n, uint32_t p, int reps, void* stream);
pm_status pm_tune_ctx(const size_t* lcs, size_t n, uint32_t p, int reps, int context, void* stream);
/* Median running time of one plan for output length lc (synchronous); in
 * PM_CTX_BATCH the time per product of a batch, as the tuner measures it
 * (kind 3 there: PM_EINVAL).
 * pm_time_plan is pm_time_plan_ctx(.., PM_CTX_SINGLE, ..). */
pm_status pm_time_plan(size_t lc, uint32_t p, const pm_plan* plan, int reps, double* us);
pm_status pm_time_plan_ctx(size_t lc, uint32_t p, const pm_plan* plan, int reps, int context, double* us);
size_t pm_tune_db_size(void);
/* Row i of the database; any output pointer may be NULL. */
pm_status pm_tune_db_get(size_t i, size_t* lc, uint32_t* p, pm_plan* plan, double* us, int* context);
pm_status pm_tune_db_add(size_t lc, uint32_t p, const pm_plan* plan, double us, int context);
void pm_tune_db_clear(void);
/* Text file, one row per line: lc p kind log_l log_ra log_rb log_c ma lq lnt us
 * context q (a line without the context is a PM_CTX_SINGLE row; q, the odd
 * factor, is required for kind 3 only).  Load appends (tuning resumes from
 * the rows already measured). */
pm_status pm_tune_db_save(const char* path);
pm_status pm_tune_db_load(const char* path);

/* ---- the learned cost model -----------------------------------------------
 * An FP32 perceptron (17 features, two tanh layers of 64, linear output)
 * predicts the log running time per relaxed coefficient of a (length, plan,
 * context); under PM_POLICY_LEARNED the plan with the least predicted time in
 * the caller's context is used (and cached).  Trained on the timing database
 * (both contexts) by the library's own forward, backward and Adam kernels.
 * The model covers the power-of-two plans (kinds 0-2): training skips the
 * database's kind-3 rows, and features or predictions of kind 3 give
 * PM_EINVAL. */
/* Feature vector (17 floats) of a (length, prime, plan, context). */
pm_status pm_model_features(size_t lc, uint32_t p, const pm_plan* plan, int context, float* out);
/* Train on the database for `steps` full-batch Adam steps at rate lr from
 * the initial weights `init` (pm_mlp_num_params() floats, host; NULL: a
 * SplitMix64-seeded Glorot-uniform draw).  losses: NULL or `steps` floats. */
pm_status pm_model_train(const float* init, int steps, float lr, float* losses);
/* Weights and target normalisation (log us per coefficient: mean, sd). */
pm_status pm_model_get(float* params, float* mean, float* sd);
pm_status pm_model_set(const float* params, float mean, float sd);
/* Predicted natural log of the running time in microseconds of n plans in a
 * context (per product in PM_CTX_BATCH). */
pm_status pm_model_predict(size_t lc, uint32_t p, const pm_plan* plans, size_t n, int context, double* log_us);
pm_status pm_model_save(const char* path);
pm_status pm_model_load(const char* path);

/* The network's kernels on host arrays (test hooks).  Parameter layout
 * W1[64][17], b1[64], W2[64][64], b2[64], W3[64], b3[1]; X is B x 17 row-major;
 * loss = mean (y - t)^2. */
size_t pm_mlp_num_params(void);
pm_status pm_mlp_forward(const float* params, const float* X, int B, float* y);
pm_status pm_mlp_loss_grad(const float* params, const float* X, const float* t, int B, float* loss, float* grads);
/* One bias-corrected Adam step (beta1 0.9, beta2 0.999, eps 1e-8) in place. */
pm_status pm_mlp_adam(float* params, const float* grads, float* m, float* v, int step, float lr);
/* `steps` Adam steps of full-batch training in place; losses: NULL or steps floats. */
pm_status pm_mlp_train(float* params, const float* X, const float* t, int B, int steps, float lr, float* losses);

/* ---- tracing ------------------------------------------------------------
 * When enabled, every kernel the library launches is bracketed by two HIP
 * events recorded on its own stream, so kernel durations can be measured in
 * a live run.  Kernel names: "direct", "lds_conv", "col_fwd", "row_conv",
 * "col_inv", "row_xform", "lds_xform", "permute", "crt", "carry_maps",
 * "carry_limbs", "widen", "patch_jobs", "mixed_split", "mixed_merge",
 * "mixed_perm", "row_jobs", "kron_pack"; a batch's graph launch is recorded as
 * "batch_graph".  While tracing is on, pm_poly_mul_batch runs its classes'
 * launches one after the other on the caller's stream instead of launching
 * its graph, so that every recorded duration is that kernel's alone. */
void pm_trace_enable(int on);
/* Forget all records (waits for the recorded events). */
void pm_trace_reset(void);
/* Total duration in ms and number of launches of `kernel` since the reset. */
pm_status pm_trace_query(const char* kernel, double* total_ms, int64_t* count);
/* Newline-separated names of the traced kernels; returns the size needed. */
size_t pm_trace_names(char* buf, size_t cap);

#ifdef __cplusplus
}
#endif
#endif
