#!/usr/bin/env python3
"""Throughput of the NTT/TFT modular polynomial product on one MI355X.

One step = one batch of 4096 independent products of uneven lengths (each
operand length log-uniform in [64, 65536], primes drawn from the four
supported ones, coefficients uniform in [0, p)), computed by one
pm_poly_mul_batch call: one hipGraph launch, plans from the learned cost
model.  value = output coefficients per second of the batched, learned-plan
path, with the inputs resident in HBM when the timed region starts.

Beside it, the same batch "plain": a loop of one pm_poly_mul call per
product with padded power-of-two plans, and the same graph with padded
default plans and with the relaxed default plans (the library without the
cost model).  The JSON line carries the roofline of the batch launch (its
algorithmic VALU slots and HBM bytes over its duration, from HIP events on
the launch stream), the dominant kernel family of the batch, and the CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P = 2013265921
G = 31                                 # a primitive root mod P
# the autotuner's picks for the two plain large products on MI355X (four-step
# L = 2^22, RA 32, RB 32, C 2^12; four-step L = 2^20, RA 16, RB 16, C 2^12,
# untruncated: at 10^6 outputs the only truncation, 31 of 32 blocks of the
# first radix 32, measured 5% slower)
TUNED_PLANS = "2,22,5,5,12,32,3,9;2,20,4,4,12,16,3,9"
CU, LANES, CLOCK = 256, 64, 2.4e9
ALU_PEAK = CU * LANES * CLOCK          # 32-bit VALU issue slots per second
HBM_PEAK = 8.0e12                      # bytes per second
# algorithmic VALU slots (gfx950: mul_hi is half rate, so it counts 2)
SLOTS_BUTTERFLY = 10                   # Shoup multiply (5) + add and subtract with range reduction (5)
SLOTS_MULMOD_CONST = 5                 # Shoup: mul_hi (2) + 2 mul_lo + sub
SLOTS_MULMOD_VAR = 8                   # Montgomery: 2 mul_hi (4) + 2 mul_lo + add + carry
MODEL = os.path.join(ROOT, "paper_1609_01010_amd", "data", "cost_model.txt")
KIND_DIRECT, KIND_LDS, KIND_FOURSTEP = 0, 1, 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nprime(plan):
    """Relaxed transform length n' = ma L / RA of a plan."""
    return plan.ma << (plan.log_l - plan.log_ra)


def per_element_slots(log_n):
    """Algorithmic VALU slots per element of n' of a product whose transforms
    span 2^log_n points: three transforms of (log_n)/2 butterflies per element,
    three four-step twiddle multiplies and the scale (constants), one
    pointwise product (variables)."""
    return 3 * (log_n / 2) * SLOTS_BUTTERFLY + 4 * SLOTS_MULMOD_CONST + SLOTS_MULMOD_VAR


def product_units(la, lb, plan):
    """(algorithmic HBM bytes, algorithmic VALU slots) of one product: operands
    read once and the result written once; a four-step plan also writes and
    reads its two n'-word intermediates (8 n' + 8 n' + 4 n' + 4 n'); the
    defining sum costs one variable product per term."""
    lc = la + lb - 1
    byts = 4 * (la + lb + lc)
    if plan.kind == KIND_DIRECT:
        return byts, SLOTS_MULMOD_VAR * la * lb
    n = nprime(plan)
    if plan.kind == KIND_FOURSTEP:
        byts += 24 * n
    return byts, n * per_element_slots(plan.log_l)


def family_units(items, plans):
    """Algorithmic (bytes, slots) per kernel family of a batch: the defining
    sums, the one-work-group convolution, and the four-step convolution's
    column forward, row and column inverse passes."""
    out = {}

    def add(k, b, s):
        x = out.setdefault(k, [0.0, 0.0])
        x[0] += b
        x[1] += s

    for it, pl in zip(items, plans):
        la, lb = it.a.size, it.b.size
        lc = la + lb - 1
        if pl.kind == KIND_DIRECT:
            add("direct", *product_units(la, lb, pl))
        elif pl.kind == KIND_LDS:
            add("lds_conv", *product_units(la, lb, pl))
        else:
            n = nprime(pl)
            log_r = pl.log_l - pl.log_c
            add("col_fwd", 4 * (la + lb) + 8 * n, 2 * n * (log_r / 2) * SLOTS_BUTTERFLY)
            add("row_conv", 12 * n, n * (3 * (pl.log_c / 2) * SLOTS_BUTTERFLY + 4 * SLOTS_MULMOD_CONST +
                                         SLOTS_MULMOD_VAR))
            add("col_inv", 4 * n + 4 * lc, n * (log_r / 2) * SLOTS_BUTTERFLY)
    return out


def row_conv_units(plan, n_rows_elems):
    """Algorithmic slots and HBM bytes of one row pass over n_rows_elems elements:
    three length-C transforms (C/2 log2 C butterflies each), three four-step
    twiddle multiplies, one pointwise product, one scaling multiply; reads two
    operands, writes one."""
    logc = plan.log_c
    per_el = 3 * (logc / 2) * SLOTS_BUTTERFLY + 4 * SLOTS_MULMOD_CONST + SLOTS_MULMOD_VAR
    return per_el * n_rows_elems, 12 * n_rows_elems


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Bytes read plus written per second by a device-to-device copy of 1 GiB
    (the attainable HBM rate the roofline fractions are also quoted against)."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = time_loop(torch, lambda i: dst.copy_(src), reps)
    del src, dst
    return 2 * nbytes / (ms * 1e-3)


def time_calls(torch, fn, reps):
    """Median milliseconds of fn() over reps runs, HIP events on the current stream."""
    import numpy as np

    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def time_loop(torch, fn, n):
    """Milliseconds per call of n back-to-back calls, HIP events on the current stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(n):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def source_hash():
    """Hash of the library sources and the shipped cost model: counter files
    taken on other sources are not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_01010_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    with open(MODEL, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def counters_from_profiles(name, src_hash):
    """A committed rocprofv3 counter summary (profiles/<name>.json), if it was
    taken on the current sources, else None."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
    except OSError:
        return None
    return d if d.get("source_sha256") == src_hash else None


# ---------------------------------------------------------------------------
# spot checks of the GPU results (the parity tests live in tests/): a
# polynomial identity at random points, evaluated here with numpy

def eval_mod(c, p, x):
    """sum_i c_i x^i mod p for coefficients c < 2^32, in blocks of 4096 powers."""
    import numpy as np

    c = np.asarray(c, dtype=np.uint64)
    B = 4096
    pw = np.empty(B, dtype=np.uint64)
    v = 1
    for i in range(B):
        pw[i] = v
        v = v * x % p
    acc, sk = 0, 1
    for k in range(0, c.size, B):
        blk = c[k:k + B]
        acc = (acc + int(((blk * pw[:blk.size]) % np.uint64(p)).sum()) % p * sk) % p
        sk = sk * v % p
    return acc


def check_product(a, b, c, p, rng, points=2, n=None, sign=0):
    """c(x) = a(x) b(x) mod p at random points x (false accept <= len(c)/p
    each); with n: the product mod x^n - sign, checked where x^n = sign."""
    for _ in range(points):
        if n is None:
            x = int(rng.integers(2, p - 1))
        else:
            root = pow(_root(p), (p - 1) // (2 * n), p)  # a primitive 2n-th root: root^n = -1
            x = pow(root, 2 * int(rng.integers(0, n)) + (0 if sign == 1 else 1), p)
        if eval_mod(c, p, x) != eval_mod(a, p, x) * eval_mod(b, p, x) % p:
            return False
    return True


def bitrev(i, bits):
    return int(format(i, f"0{bits}b")[::-1], 2)


def limbs_value(limbs):
    import numpy as np

    return int.from_bytes(np.asarray(limbs, dtype="<u2").tobytes(), "little")


# ---------------------------------------------------------------------------
# CPU baselines

def cpu_baseline(items, target_s=10.0):
    """The oracle timed on a bounded sample of the batch: its schoolbook sum
    c_k = sum a_i b_(k-i) mod p on output coefficients drawn uniformly over
    all the batch's outputs, and its textbook radix-2 transforms on every
    16th product whole."""
    import numpy as np

    from oracle import poly as op

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    rng = np.random.default_rng(7)
    lcs = np.array([it.a.size + it.b.size - 1 for it in items], dtype=np.int64)
    cum = np.cumsum(lcs)
    total = int(cum[-1])

    def run(n):
        picks = np.sort(rng.choice(total, size=n, replace=False))
        prod = np.searchsorted(cum, picks, side="right")
        t0 = time.perf_counter()
        for k in np.unique(prod):
            ks = picks[prod == k] - (cum[k] - lcs[k])
            it = items[int(k)]
            op.poly_mul_sample(it.a, it.b, it.p, ks)
        return time.perf_counter() - t0

    run(256)  # loads the oracle's C library and starts its threads
    # grow the sample until it takes about target_s (at most 8 M coefficients)
    n, cap = 4096, 8_000_000
    dt = run(n)
    while dt < 0.5 * target_s and n < cap:
        n = int(min(cap, n * min(target_s / max(dt, 1e-3), 50.0)))
        dt = run(n)
    sub = items[::16]
    t0 = time.perf_counter()
    for it in sub:
        op.poly_mul_ntt(it.a, it.b, it.p, _root(it.p))
    dt_ntt = time.perf_counter() - t0
    lc_sub = sum(it.a.size + it.b.size - 1 for it in sub)
    return {
        "value": n / dt,
        "unit": "coeffs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} output coefficients drawn uniformly over the {len(items)} products' {total} outputs, by "
                  f"the oracle's schoolbook sum c_k = sum a_i b_(k-i) mod p (OpenMP over k); {dt:.1f} s",
        "ntt_route": {"value": lc_sub / dt_ntt, "unit": "coeffs/s", "cores": threads,
                      "sample": f"every 16th product ({len(sub)} of {len(items)}) whole by the oracle's radix-2 "
                                f"transforms; {dt_ntt:.2f} s"},
    }


def _root(p):
    from paper_1609_01010_amd import inputs

    return inputs.PRIMES[p]


# ---------------------------------------------------------------------------
# the headline: the 4096-product batch

def padded_plan(pm, lc, p):
    """The default plan of output length lc without truncation (the padded
    power-of-two transform); the defining sum for at most 64 outputs."""
    pl = pm.plan_for(lc, p)
    if pl.kind != KIND_DIRECT:
        pl.ma = 1 << pl.log_ra
    return pl


def batch_bench(pm, torch, dev, args):
    import ctypes

    import numpy as np

    from paper_1609_01010_amd import inputs

    items = inputs.batch_uneven()
    lcs = [it.a.size + it.b.size - 1 for it in items]
    ncoef = sum(lcs)
    # two buffer sets (each about 0.9 GB of operands and outputs), alternated
    # from step to step: every step reads its inputs from HBM, not from the
    # 256 MB MALL
    sets = []
    for _ in range(2):
        probs = [(torch.from_numpy(it.a).to(dev), torch.from_numpy(it.b).to(dev), it.p) for it in items]
        outs = [torch.empty(lc, dtype=torch.uint32, device=dev) for lc in lcs]
        sets.append((probs, outs))
    torch.cuda.synchronize()
    set_bytes = sum(4 * (it.a.size + it.b.size + lc) for it, lc in zip(items, lcs))
    log(f"batch: {len(items)} products, {ncoef} output coefficients, {set_bytes / 1e9:.2f} GB per buffer set")

    # --- batched + learned plans (the headline)
    pm.model_load(MODEL)
    pm.set_policy(pm.POLICY_LEARNED)
    pm.plan_cache_clear()
    prepared = [pm.PreparedBatch(pr, outs=o) for pr, o in sets]
    t0 = time.perf_counter()
    prepared[0].run()  # plans the shape: the model's picks, checked against the default plans on the whole batch
    torch.cuda.synchronize()
    first_call_s = time.perf_counter() - t0
    plans = pm.batch_plans_used(len(items))
    for i in range(args.warmup):
        prepared[i % 2].run()
    torch.cuda.synchronize()
    if pm.stream_check() != 0:
        raise SystemExit("device reported an error during warm-up")
    # spot check: 24 products of each buffer set run so far at two random points
    rng = np.random.default_rng(5)
    sets_run = sorted({0} | {i % 2 for i in range(args.warmup)})
    for k in rng.choice(len(items), 24, replace=False):
        for si in sets_run:
            it = items[int(k)]
            assert check_product(it.a, it.b, sets[si][1][int(k)].cpu().numpy(), it.p, rng), "wrong batch product"

    # timed: K graph launches back to back, HIP events on the launch stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        prepared[i % 2].run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = e0.elapsed_time(e1)
    ms_step = gpu_ms / args.steps
    if pm.stream_check() != 0:
        raise SystemExit("device reported an error in the timed steps")

    # per-kernel durations: the same batch traced (its classes' launches one
    # after the other, each bracketed by its own events)
    pm.trace_reset()
    pm.trace_enable(True)
    for i in range(2):
        prepared[i % 2].run()
    torch.cuda.synchronize()
    pm.trace_enable(False)
    traced = {}
    for name in pm.trace_names():
        tot, n = pm.trace_query(name)
        traced[name] = {"launches": n, "total_us_per_batch": 1e3 * tot / 2, "avg_us": 1e3 * tot / max(n, 1)}
    pm.trace_reset()
    traced_ms = sum(v["total_us_per_batch"] for v in traced.values()) / 1e3

    fam = family_units(items, plans)
    for name, v in traced.items():
        if name in fam:
            v["alg_bytes_per_batch"], v["alg_slots_per_batch"] = fam[name]
            t = v["total_us_per_batch"] * 1e-6
            v["alu_frac"] = fam[name][1] / t / ALU_PEAK
            v["hbm_frac"] = fam[name][0] / t / HBM_PEAK
    dom = max((k for k in traced if k in fam), key=lambda k: traced[k]["total_us_per_batch"])
    plan_hist = {}
    for pl in plans:
        key = ",".join(str(v) for v in pl.as_tuple()[:5]) + "," + ",".join(str(v) for v in pl.as_tuple()[6:])
        plan_hist[key] = plan_hist.get(key, 0) + 1

    byts, slots = 0.0, 0.0
    for it, pl in zip(items, plans):
        b, s_ = product_units(it.a.size, it.b.size, pl)
        byts += b
        slots += s_
    res = {
        "items": items, "plans": plans, "ncoef": ncoef, "ms_step": ms_step, "gpu_ms": gpu_ms, "wall": wall,
        "value": ncoef / (ms_step * 1e-3), "alg_bytes": byts, "alg_slots": slots,
        "traced": traced, "traced_ms": traced_ms, "dom": dom, "plan_hist": plan_hist,
        "first_call_s": first_call_s, "set_bytes": set_bytes, "plain": None,
    }
    if args.headline_only:
        pm.set_policy(pm.POLICY_DEFAULT)
        return res

    # --- plain: one call per product, padded power-of-two plans
    pm.set_policy(pm.POLICY_DEFAULT)
    pm.plan_cache_clear()
    pplans = [padded_plan(pm, lc, it.p) for it, lc in zip(items, lcs)]
    L = pm.lib()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    probs0, outs0 = sets[0]
    args_loop = [(ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(y.data_ptr()), y.numel(), pp,
                  ctypes.c_void_p(o.data_ptr()), ctypes.byref(pl), sp)
                 for (x, y, pp), o, pl in zip(probs0, outs0, pplans)]

    def plain_loop():
        for a_ in args_loop:
            st = L.pm_poly_mul_plan(*a_)
            if st:
                raise SystemExit(f"pm_poly_mul_plan failed: {st}")

    plain_loop()
    ms_loop = time_calls(torch, plain_loop, 3)

    def graph_time(put_plans):
        pm.plan_cache_clear()
        if put_plans is not None:
            for it, lc, pl in zip(items, lcs, put_plans):
                if pl.kind != KIND_DIRECT:
                    pm.plan_cache_put(lc, it.p, pl)
        pb = [pm.PreparedBatch(pr, outs=o) for pr, o in sets]
        pb[0].run()
        torch.cuda.synchronize()
        ms = time_calls(torch, lambda: (pb[0].run(), pb[1].run()), max(5, args.steps // 4)) / 2
        return ms

    ms_graph_padded = graph_time(pplans)
    ms_graph_default = graph_time(None)
    pm.plan_cache_clear()
    if pm.stream_check() != 0:
        raise SystemExit("device error in the plain legs")
    # the last leg (relaxed default plans) left its products in set 0: check some
    for k in rng.choice(len(items), 8, replace=False):
        it = items[int(k)]
        assert check_product(it.a, it.b, sets[0][1][int(k)].cpu().numpy(), it.p, rng), "wrong batch product"
    pad_bytes, pad_slots = 0.0, 0.0
    for it, pl in zip(items, pplans):
        b, s = product_units(it.a.size, it.b.size, pl)
        pad_bytes += b
        pad_slots += s

    res["plain"] = {
        "loop_of_single_calls_padded_ms": ms_loop,
        "graph_padded_default_plans_ms": ms_graph_padded,
        "graph_relaxed_default_plans_ms": ms_graph_default,
        "batched_learned_ms": ms_step,
        "speedup_vs_loop_padded": ms_loop / ms_step,
        "speedup_vs_graph_padded": ms_graph_padded / ms_step,
        "speedup_vs_graph_default": ms_graph_default / ms_step,
        "padded_alg_slots": pad_slots, "padded_alg_bytes": pad_bytes,
        "note": "loop: one pm_poly_mul_plan call per product (host-call bound); graph legs: the same "
                "pm_poly_mul_batch graph with padded power-of-two default plans, and with the relaxed "
                "default plans (the library without the cost model)",
    }
    del sets, prepared
    return res


# ---------------------------------------------------------------------------
# the other workloads

def standalone_transform(pm, torch, dev, copy_bw, n_calls=40):
    """Forward transform of 2^22 points in bit-reversed order (the TFT hook with
    n = L): two passes over HBM, 16 N algorithmic bytes; 8 rotating buffer
    pairs (256 MiB); four outputs checked against direct evaluation."""
    from paper_1609_01010_amd import inputs

    N = 1 << 22
    out = {}
    for pp in (2013265921, 998244353):
        g = inputs.PRIMES[pp]
        # 16 inputs and 16 outputs of 16 MiB each (512 MiB, twice the MALL),
        # rotated, so every transform reads and writes HBM
        nb = 16
        xs = [torch.from_numpy(inputs.uniform_mod(inputs.rng_for((140, pp % 1000, k)), N, pp)).to(dev)
              for k in range(nb)]
        ys = [torch.empty(N, dtype=torch.uint32, device=dev) for _ in range(nb)]

        def fwd(i):
            pm.tft(xs[i % nb], N, N, pp, out=ys[i % nb])

        for i in range(nb):
            fwd(i)
        ms = time_loop(torch, fwd, n_calls)
        pm.trace_reset()
        pm.trace_enable(True)
        for i in range(nb):
            fwd(i)
        torch.cuda.synchronize()
        pm.trace_enable(False)
        kern = {}
        for name in pm.trace_names():
            tot, n = pm.trace_query(name)
            kern[name] = 1e3 * tot / max(n, 1)
        pm.trace_reset()
        x0, y0 = xs[0].cpu().numpy(), ys[0].cpu().numpy()
        w = pow(g, (pp - 1) // N, pp)
        ok = all(int(y0[i]) == eval_mod(x0, pp, pow(w, bitrev(i, 22), pp)) for i in (0, 1, 12345, N - 1))
        out[f"ntt_2^22_p{pp}"] = {"us": ms * 1e3, "points_per_s": N / (ms * 1e-3),
                                  "hbm_alg_GBps": 16 * N / (ms * 1e-3) / 1e9,
                                  "hbm_frac": 16 * N / (ms * 1e-3) / HBM_PEAK,
                                  "hbm_frac_vs_copy": 16 * N / (ms * 1e-3) / copy_bw,
                                  "kernels_avg_us": kern,
                                  "checked_at_random_points": bool(ok)}
        del xs, ys
    return out


def int_product(pm, torch, dev, reps=5):
    """The three-primes product of two 2^21-limb integers (config 3), with
    both digit sizes; per-kernel durations from a traced call."""
    from paper_1609_01010_amd import inputs

    out = {}
    # the three-primes product of two 2^21-limb integers: pm_int_mul's own
    # choice (32-bit digits, 2^21-point transforms), and the 16-bit limbs as
    # digits (2^22-point transforms)
    ia, ib = inputs.int_operands()
    tia, tib = torch.from_numpy(ia).to(dev), torch.from_numpy(ib).to(dev)
    ic = torch.empty(ia.size + ib.size, dtype=torch.uint16, device=dev)
    q = (1 << 61) - 1
    want = (limbs_value(ia) % q) * (limbs_value(ib) % q) % q
    # one call of each digit size first: the stream's workspace is then sized
    # for both before anything is timed
    for digits in (16, None):
        pm.int_mul(tia, tib, out=ic, digits=digits)
    torch.cuda.synchronize()
    for key, digits in (("int_mul_2^21x2^21_limbs", None), ("int_mul_2^21x2^21_limbs_digits16", 16)):
        pm.int_mul(tia, tib, out=ic, digits=digits)
        ms = time_calls(torch, lambda: pm.int_mul(tia, tib, out=ic, digits=digits), reps)
        pm.trace_reset()
        pm.trace_enable(True)
        pm.int_mul(tia, tib, out=ic, digits=digits)
        torch.cuda.synchronize()
        pm.trace_enable(False)
        ik = {}
        for name in pm.trace_names():
            tot, n = pm.trace_query(name)
            ik[name] = 1e3 * tot
        pm.trace_reset()
        got = ic.cpu().numpy()
        ok = limbs_value(got) % q == want
        out[key] = {"digits": "32-bit (pairs of limbs), 2^21-point transforms" if digits is None
                    else "16-bit limbs, 2^22-point transforms",
                    "ms": ms, "limbs_per_s": got.size / (ms * 1e-3), "kernels_us": ik,
                    "check": "product mod 2^61-1 matches" if ok else "MISMATCH"}
    del tia, tib, ic
    return out


def large_products(pm, torch, dev, args):
    """The two plain large products over Z/2013265921Z (2^21 x 2^21 through
    L = 2^22, and 600001 x 400000 with 10^6 outputs through L = 2^20), with
    the autotuner's plans; per-kernel durations from a traced pass and
    the row pass's roofline."""
    import numpy as np

    from paper_1609_01010_amd import inputs

    a2, b2, _ = inputs.large_pow2_product()
    a3, b3, _ = inputs.large_tft_product()
    lc2, lc3 = a2.size + b2.size - 1, a3.size + b3.size - 1
    sets = []
    for _ in range(16):
        sets.append(tuple(torch.from_numpy(x).to(dev) for x in (a2, b2, a3, b3)) +
                    (torch.empty(lc2, dtype=torch.uint32, device=dev), torch.empty(lc3, dtype=torch.uint32, device=dev)))
    plan2, plan3 = (pm.Plan(*[int(v) for v in s.split(",")]) for s in args.plans.split(";"))

    def step(i):
        ta2, tb2, ta3, tb3, c2, c3 = sets[i % len(sets)]
        pm.poly_mul(ta2, tb2, P, out=c2, plan=plan2)
        pm.poly_mul(ta3, tb3, P, out=c3, plan=plan3)

    for i in range(3):
        step(i)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    assert check_product(a2, b2, sets[0][4].cpu().numpy(), P, rng)
    assert check_product(a3, b3, sets[0][5].cpu().numpy(), P, rng)
    n = 30
    ms = time_loop(torch, step, n)
    pm.trace_reset()
    pm.trace_enable(True)
    for i in range(n):
        step(i)
    torch.cuda.synchronize()
    pm.trace_enable(False)
    kernels = {}
    for name in pm.trace_names():
        tot, k = pm.trace_query(name)
        kernels[name] = {"launches": k, "avg_us": 1e3 * tot / max(k, 1)}
    pm.trace_reset()
    row = kernels["row_conv"]
    slots2, bytes2 = row_conv_units(plan2, (plan2.ma << plan2.log_rb) << plan2.log_c)
    slots3, bytes3 = row_conv_units(plan3, (plan3.ma << plan3.log_rb) << plan3.log_c)
    achieved = (slots2 + slots3) / 2 / (row["avg_us"] * 1e-6)
    del sets
    return {
        "workload": "2^21 x 2^21 (transform 2^22) + 600001 x 400000 (10^6 outputs, transform 2^20) mod 2013265921",
        "plans": [list(plan2.as_tuple()), list(plan3.as_tuple())],
        "us_per_step": ms * 1e3, "coeffs_per_s": (lc2 + lc3) / (ms * 1e-3),
        "kernels": kernels,
        "row_conv_alu_frac": achieved / ALU_PEAK,
        "row_conv_hbm_frac": (bytes2 + bytes3) / 2 / (row["avg_us"] * 1e-6) / HBM_PEAK,
    }


def extra_configs(pm, torch, dev, copy_bw, args, reps=5):
    """The other workloads, each timed on its own: the 1024 x 1024 product
    (latency, beside its kernel time), the two plain large products, the
    three-primes integer product, the 2^22-point transform, a bivariate
    product, the products of the two factor rings of eq. 13 and the general
    radix."""
    import numpy as np

    from paper_1609_01010_amd import inputs

    out = {}
    rng = np.random.default_rng(8)
    pm.set_policy(pm.POLICY_DEFAULT)
    pm.plan_cache_clear()
    a, b, p = inputs.single_product_1024()
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    c = torch.empty(2047, dtype=torch.uint32, device=dev)
    pm.poly_mul(ta, tb, p, out=c)
    ms = time_calls(torch, lambda: pm.poly_mul(ta, tb, p, out=c), 50)
    ms_loop = time_loop(torch, lambda i: pm.poly_mul(ta, tb, p, out=c), 200)
    pm.trace_reset()
    pm.trace_enable(True)
    for _ in range(20):
        pm.poly_mul(ta, tb, p, out=c)
    torch.cuda.synchronize()
    pm.trace_enable(False)
    ktot = 0.0
    for name in pm.trace_names():
        tot, n = pm.trace_query(name)
        ktot += 1e3 * tot / 20
    pm.trace_reset()
    t0 = time.perf_counter()
    for _ in range(200):
        pm.poly_mul(ta, tb, p, out=c)
    host_us = (time.perf_counter() - t0) / 200 * 1e6
    torch.cuda.synchronize()
    assert check_product(a, b, c.cpu().numpy(), p, rng, points=3)
    out["single_1024x1024_p998244353"] = {
        "us_one_call": ms * 1e3, "us_per_call_back_to_back": ms_loop * 1e3, "kernel_us": ktot,
        "host_us_per_call": host_us, "coeffs_per_s": 2047 / (ms * 1e-3), "checked_at_random_points": True}

    out["plain_large_products"] = large_products(pm, torch, dev, args)

    out.update(int_product(pm, torch, dev, reps))

    out.update(standalone_transform(pm, torch, dev, copy_bw))

    # a bivariate product by Kronecker substitution: 1024 x 1024 coefficients
    # times 1024 x 1024 (2047^2 outputs, one 2^22 transform)
    rng = inputs.rng_for(141)
    ma = torch.from_numpy(inputs.uniform_mod(rng, 1 << 20, 2013265921).reshape(1024, 1024)).to(dev)
    mb = torch.from_numpy(inputs.uniform_mod(rng, 1 << 20, 2013265921).reshape(1024, 1024)).to(dev)
    mc = torch.empty((2047, 2047), dtype=torch.uint32, device=dev)
    pm.poly_mul_multi(ma, mb, 2013265921, out=mc)
    ms = time_loop(torch, lambda i: pm.poly_mul_multi(ma, mb, 2013265921, out=mc), 20)
    out["bivariate_1024^2_x_1024^2_p2013265921"] = {"us": ms * 1e3, "coeffs_per_s": 2047 * 2047 / (ms * 1e-3)}
    del ma, mb, mc

    # products in the two factors of eq. 13 at n = 2^21 (length-n transforms, no padding)
    a2, b2, pp = inputs.large_pow2_product()
    n21 = a2.size
    ra, rb = torch.from_numpy(a2).to(dev), torch.from_numpy(b2).to(dev)
    rc = torch.empty(n21, dtype=torch.uint32, device=dev)
    for name, fn in (("cyclic", pm.cyclic_mul), ("negacyclic", pm.negacyclic_mul)):
        fn(ra, rb, n21, pp, out=rc)
        ms = time_loop(torch, lambda i: fn(ra, rb, n21, pp, out=rc), 20)
        ok = check_product(a2, b2, rc.cpu().numpy(), pp, rng, n=n21, sign=1 if name == "cyclic" else -1)
        out[f"{name}_2^21_p{pp}"] = {"us": ms * 1e3, "coeffs_per_s": n21 / (ms * 1e-3), "checked_at_random_points": bool(ok)}
    del ra, rb, rc
    # general radix: products of length q 2^k - 1 through the length-q 2^k
    # circular convolution (prime-factor split), beside the default
    # power-of-two plan (relaxed TFT) of the same product
    for q, k in ((3, 20), (5, 18), (15, 16)):
        la = (q << k) // 2
        lb = (q << k) - la
        ma_, mb_ = inputs.poly_pair((163, q), la, lb, pp)
        lcm = la + lb - 1
        xa, xb = torch.from_numpy(ma_).to(dev), torch.from_numpy(mb_).to(dev)
        xc = torch.empty(lcm, dtype=torch.uint32, device=dev)
        pm.poly_mul_mixed(xa, xb, pp, q, out=xc)
        ms_mixed = time_loop(torch, lambda i: pm.poly_mul_mixed(xa, xb, pp, q, out=xc), 20)
        ok = check_product(ma_, mb_, xc.cpu().numpy(), pp, rng)
        pm.poly_mul(xa, xb, pp, out=xc)
        ms_pow2 = time_loop(torch, lambda i: pm.poly_mul(xa, xb, pp, out=xc), 20)
        out[f"mixed_radix_{q}x2^{k}_p{pp}"] = {
            "lc": lcm, "us": ms_mixed * 1e3, "coeffs_per_s": lcm / (ms_mixed * 1e-3),
            "pow2_default_us": ms_pow2 * 1e3, "checked_at_random_points": bool(ok)}
        del xa, xb, xc
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the batched, learned-plan steps (no plain legs, other workloads or CPU baseline): "
                         "the command the profiles of the batch are taken with")
    ap.add_argument("--plans", default=TUNED_PLANS,
                    help="plans of the two plain large products among the other workloads, "
                         "'kind,log_l,log_ra,log_rb,log_c,ma,lq,lnt;...' (default: the autotuner's picks on MI355X)")
    ap.add_argument("--large-only", action="store_true",
                    help="only the two plain large products with --plans (the command their profiles are taken "
                         "with); prints their timings, not the headline line")
    ap.add_argument("--transform-only", action="store_true",
                    help="only the forward transforms of 2^22 points (the command their counters are taken with); "
                         "prints their timings, not the headline line")
    ap.add_argument("--int-only", action="store_true",
                    help="only the three-primes integer product of two 2^21-limb integers, both digit sizes (the "
                         "command its profile is taken with); prints its timings, not the headline line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 256 MiB three times (reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        src = torch.empty(1 << 26, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library's path runs on a single MI355X and has no "
              "multi-GPU mode. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_01010_amd as pm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    pm.lib()
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    copy_bw = copy_bandwidth(torch, dev)
    if args.transform_only:
        print(json.dumps(standalone_transform(pm, torch, dev, copy_bw)), flush=True)
        return
    if args.large_only:
        print(json.dumps(large_products(pm, torch, dev, args)), flush=True)
        return
    if args.int_only:
        print(json.dumps(int_product(pm, torch, dev)), flush=True)
        return

    if args.headline_only:
        args.no_cpu_baseline = args.no_extra = True
    r = batch_bench(pm, torch, dev, args)
    t = r["ms_step"] * 1e-3
    src_hash = source_hash()
    counters = counters_from_profiles("batch_counters.json", src_hash)
    traffic = counters.get("hbm_bytes_per_batch") if counters else None
    dom = r["dom"]
    dk = r["traced"][dom]
    roofline = {
        "kernel": "one pm_poly_mul_batch graph launch: every kernel of the 4096 products",
        "bound": "alu",
        "achieved": r["alg_slots"] / t / 1e12,
        "peak": ALU_PEAK / 1e12,
        "unit": "Tslot/s",
        "frac": r["alg_slots"] / t / ALU_PEAK,
        "traffic": traffic,
        "algorithmic_slots_per_launch": r["alg_slots"],
        "algorithmic_bytes_per_launch": r["alg_bytes"],
        "launch_us": r["ms_step"] * 1e3,
        "hbm_achieved_GBps": r["alg_bytes"] / t / 1e9,
        "hbm_frac": r["alg_bytes"] / t / HBM_PEAK,
        "hbm_frac_vs_copy": r["alg_bytes"] / t / copy_bw,
        "copy_GBps": copy_bw / 1e9,
        "dominant_kernel": {
            "family": dom, "launches_per_batch": dk["launches"] / 2, "total_us_per_batch": dk["total_us_per_batch"],
            "bound": "alu", "achieved": dk["alg_slots_per_batch"] / (dk["total_us_per_batch"] * 1e-6) / 1e12,
            "peak": ALU_PEAK / 1e12, "unit": "Tslot/s", "frac": dk["alu_frac"], "hbm_frac": dk["hbm_frac"],
            "timing": "the batch's class launches run one after the other, each between its own HIP events",
        },
        "slot_model": f"{SLOTS_BUTTERFLY} slots per radix-2 butterfly, {SLOTS_MULMOD_CONST} per multiply by a "
                      f"constant, {SLOTS_MULMOD_VAR} per product of two variables; (15 log2 L + 28) n' per product",
    }
    cpu = None if args.no_cpu_baseline else cpu_baseline(r["items"])
    extra = None
    if not args.no_extra:
        torch.cuda.empty_cache()
        extra = extra_configs(pm, torch, dev, copy_bw, args)
    out = {
        "metric": "conv coefficients/s",
        "value": r["value"],
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "batched + learned plans: 4096 independent products, operand lengths log-uniform in "
                        "[64, 65536], primes uniform over 998244353, 2013265921, 469762049, 167772161, "
                        "one pm_poly_mul_batch call (one hipGraph launch)",
            "coeffs_per_step": r["ncoef"],
            "buffer_sets": 2,
            "bytes_per_buffer_set": r["set_bytes"],
            "plans_used": r["plan_hist"],
            "plan_source": "the shipped cost model (data/cost_model.txt) in the batch context, one plan family per "
                           "transform length and prime, kept for the shape only if the whole batch ran faster "
                           "with them than with the default plans on its first call",
            "first_call_s": r["first_call_s"],
            "wall_s": r["wall"],
        },
        "roofline": roofline,
        "plain": r["plain"],
        "cpu_baseline": cpu,
        "kernels": r["traced"],
        "other_configs": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
