"""Parity of the HIP path with the CPU oracle, element by element, through the C ABI.

Bit-exact everywhere: the method computes in exact modular integers.
"""

import random
import sys

import numpy as np
import pytest

from oracle import poly as op
from paper_1609_01010_amd import inputs

pytestmark = pytest.mark.gpu

PRIMES = list(inputs.PRIMES.items())


def dev(x, dtype=np.uint32):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=dtype))).cuda()


def host(t):
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _product(pm, a, b, p, plan=None):
    c = pm.poly_mul(dev(a), dev(b), p, plan=plan)
    assert pm.stream_check() == 0
    return host(c)


def test_single_product_1024(gpu_lib):
    """1024 x 1024 coefficients mod 998244353: size-2048 transforms (one work-group)."""
    pm = gpu_lib
    a, b, p = inputs.single_product_1024()
    say("case: 1024x1024 p=998244353")
    got = _product(pm, a, b, p)
    assert got.shape == (2047,)
    assert np.array_equal(got, op.poly_mul(a, b, p))


@pytest.mark.parametrize("p,g", PRIMES)
def test_products_across_plan_kinds(gpu_lib, p, g):
    """Defining sum, one-work-group and four-step plans, ragged tails, TFT truncation."""
    pm = gpu_lib
    shapes = [(1, 1), (1, 7), (5, 3), (33, 32), (40, 25), (64, 3), (65, 64), (100, 29), (127, 2), (700, 349),
              (1024, 1025), (3000, 1777), (4097, 4096), (8192, 8193), (9000, 7001), (16385, 3), (20000, 12769),
              (40000, 33000), (65536, 65536), (131072, 1)]
    for i, (la, lb) in enumerate(shapes):
        say("case:", p, la, lb)
        a, b = inputs.poly_pair((100, i, p % 997), la, lb, p)
        got = _product(pm, a, b, p)
        assert np.array_equal(got, op.poly_mul(a, b, p)), (la, lb, p)


def test_edge_values(gpu_lib):
    pm = gpu_lib
    for p, _ in PRIMES:
        for la, lb in ((1, 1), (300, 200), (5000, 4000), (20000, 30000)):
            say("case: extreme", p, la, lb)
            for fill_a, fill_b in ((p - 1, p - 1), (0, 5), (1, p - 1)):
                a = np.full(la, fill_a, dtype=np.uint32)
                b = np.full(lb, fill_b, dtype=np.uint32)
                got = _product(pm, a, b, p)
                assert np.array_equal(got, op.poly_mul(a, b, p))


def test_every_candidate_plan_agrees(gpu_lib):
    """Plan invariance: every plan of the tuner's space returns the same product."""
    pm = gpu_lib
    for p in (998244353, 2013265921):
        for lc in (129, 2047, 5000, 17000, 70000, 300001):
            la, lb = inputs.split_output_length(lc)
            a, b = inputs.poly_pair((101, lc), la, lb, p)
            want = op.poly_mul(a, b, p)
            for P in pm.plan_candidates(lc, p):
                say("case: plan", p, lc, P)
                got = _product(pm, a, b, p, plan=P)
                assert np.array_equal(got, want), (p, lc, P)


def test_operand_half_length_boundary(gpu_lib):
    """An operand of at most L/2 values leaves the upper half of every forward
    column zero and takes the shortened first level; one value more does not.
    Every candidate plan of L = 2^16 on both sides of that boundary, with the
    extreme value p - 1 at the last position of each operand."""
    pm = gpu_lib
    L = 1 << 16
    for p in (998244353, 2013265921):
        for la in (L // 2, L // 2 + 1):
            lb = L - la  # lc = L - 1
            a, b = inputs.poly_pair((103, la, p % 1000), la, lb, p)
            a[-1] = p - 1
            b[-1] = p - 1
            want = op.poly_mul(a, b, p)
            for P in pm.plan_candidates(L - 1, p):
                say("case: half boundary", p, la, P)
                got = _product(pm, a, b, p, plan=P)
                assert np.array_equal(got, want), (p, la, P)


@pytest.mark.parametrize("p", [998244353, 2013265921])
def test_truncated_inverse_near_full(gpu_lib, p):
    """Relaxed plans that keep all but d = 0..4 blocks of the first radix
    (RA = 8, 16, 32): the truncated inverse completes the d missing values
    from the known ones for d <= 3 and runs the recursion for d = 4; every
    kernel family (one work-group, four-step with and without a second
    column radix) against the schoolbook oracle."""
    pm = gpu_lib
    seen = set()
    for logL in (11, 13, 16):
        L = 1 << logL
        for lra in (3, 4, 5):
            RA = 1 << lra
            for d in range(5):
                lc = (RA - d) * (L // RA) - 3  # needs RA - d blocks of L / RA
                la, lb = inputs.split_output_length(lc)
                a, b = None, None
                for P in pm.plan_candidates(lc, p):
                    if P.kind == 0 or P.log_ra != lra or P.ma != RA - d:
                        continue
                    fam = (P.kind, P.log_rb > 0, lra, d)
                    if fam in seen:
                        continue
                    seen.add(fam)
                    if a is None:
                        a, b = inputs.poly_pair((103, lc, p % 1000), la, lb, p)
                        want = op.poly_mul(a, b, p)
                    say("case: near-full truncation", p, lc, P)
                    assert np.array_equal(_product(pm, a, b, p, plan=P), want), (p, lc, P)
    # every family and d <= 3 reached: one work-group, and four-step with RB = 1
    # and with RB > 1 (which needs RA >= 16)
    for fam in ((1, False), (2, False), (2, True)):
        for lra in (3, 4, 5):
            if fam == (2, True) and lra < 4:
                continue
            for d in range(4):
                assert (fam + (lra, d)) in seen, (fam, lra, d)


def test_large_power_of_two_product_sampled(gpu_lib):
    """2^21 x 2^21 mod 2013265921 (transform 2^22): sampled coefficients by the
    defining sum, 16 random points by evaluation."""
    pm = gpu_lib
    a, b, p = inputs.large_pow2_product()
    say("case: 2^21 x 2^21 p=2013265921")
    got = _product(pm, a, b, p)
    assert got.size == (1 << 22) - 1
    rng = random.Random(1)
    ks = sorted(set([0, 1, 2, (1 << 21) - 1, 1 << 21, got.size - 2, got.size - 1] +
                    rng.sample(range(got.size), 300)))
    assert np.array_equal(got[ks], op.poly_mul_sample(a, b, p, ks))
    for _ in range(16):
        x = rng.randrange(p)
        assert op.eval_at(got, p, x) == op.eval_at(a, p, x) * op.eval_at(b, p, x) % p
    # and the full array against the textbook transform route
    assert np.array_equal(got, op.poly_mul_ntt(a, b, p, 31))


def test_maximum_sizes(gpu_lib):
    """The largest transform lengths the library accepts: L = 2^24 mod
    2013265921 (the library's limit) and L = 2^23 mod 998244353 (its 2-adic
    order), the integer product at na + nb - 1 = 2^23, and the transform of
    2^24 points.  Sampled coefficients against the defining sum, the product
    at random points, the integer product mod 2^61 - 1, the transform against
    the evaluation definition and its exact round trip."""
    pm = gpu_lib
    rng = random.Random(24)
    for p, lg in ((2013265921, 23), (998244353, 22)):
        say("case: maximum product", p, lg)
        a, b = inputs.poly_pair((104, lg), 1 << lg, 1 << lg, p)
        got = host(pm.poly_mul(dev(a), dev(b), p))
        assert pm.stream_check() == 0
        assert got.size == (1 << (lg + 1)) - 1
        ks = sorted(set([0, 1, got.size // 2, got.size - 1] + rng.sample(range(got.size), 28)))
        assert np.array_equal(got[ks], op.poly_mul_sample(a, b, p, ks))
        for _ in range(4):
            x = rng.randrange(2, p)
            assert op.eval_at(got, p, x) == op.eval_at(a, p, x) * op.eval_at(b, p, x) % p
    ia, ib = inputs.int_operands(1 << 22, tag=105)
    q = (1 << 61) - 1
    want = (op.limbs_to_int(ia) % q) * (op.limbs_to_int(ib) % q) % q
    for digits in (32, 16):
        say("case: maximum integer product, digits", digits)
        ic = host(pm.int_mul(dev(ia, np.uint16), dev(ib, np.uint16), digits=digits))
        assert pm.stream_check() == 0
        assert op.limbs_to_int(ic) % q == want, digits
        assert ic.size == 1 << 23
    say("case: transform of 2^24 points")
    p, g = 2013265921, inputs.PRIMES[2013265921]
    x = inputs.uniform_mod(inputs.rng_for(106), 1 << 24, p)
    X = host(pm.ntt(dev(x), p))
    ks = [0, 1, 12345, (1 << 24) - 1]
    assert np.array_equal(X[ks], op.dft_eval(x, p, g, ks=ks))
    assert np.array_equal(host(pm.ntt(dev(X), p, inverse=True)), x)
    assert pm.stream_check() == 0


def test_large_tft_product(gpu_lib):
    """600001 x 400000 mod 2013265921 -> 10^6 coefficients by a truncated transform."""
    pm = gpu_lib
    a, b, p = inputs.large_tft_product()
    P = pm.plan_for(1000000, p)
    assert (P.ma << (P.log_l - P.log_ra)) < (1 << 20), "must not pad to 2^20"
    say("case: 600001 x 400000 p=2013265921", P)
    got = _product(pm, a, b, p)
    assert got.size == 1000000
    assert np.array_equal(got, op.poly_mul_ntt(a, b, p, 31))
    rng = random.Random(2)
    ks = sorted(rng.sample(range(got.size), 200))
    assert np.array_equal(got[ks], op.poly_mul_sample(a, b, p, ks))


def test_large_products_with_the_bench_plans(gpu_lib):
    """The two plain large products in the launch configuration bench.py
    times (its plans, pinned per call): 2^21 x 2^21 and 600001 x 400000 mod
    2013265921, whole arrays against the oracle's transform route."""
    import importlib.util
    import os

    pm = gpu_lib
    spec = importlib.util.spec_from_file_location(
        "bench_plans", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    plans = [pm.Plan(*[int(v) for v in t.split(",")]) for t in bench.TUNED_PLANS.split(";")]
    for (a, b, p), plan in zip((inputs.large_pow2_product(), inputs.large_tft_product()), plans):
        say("case: bench plan", plan.as_tuple(), a.size, b.size)
        got = _product(pm, a, b, p, plan=plan)
        assert got.size == a.size + b.size - 1
        assert np.array_equal(got, op.poly_mul_ntt(a, b, p, 31)), plan.as_tuple()


@pytest.mark.parametrize("p,g", PRIMES)
def test_ntt_hook(gpu_lib, p, g):
    pm = gpu_lib
    for logn in (1, 2, 5, 6, 10, 11, 14, 15, 16, 20):
        n = 1 << logn
        say("case: ntt", p, n)
        x = inputs.uniform_mod(inputs.rng_for((102, logn)), n, p)
        X = host(pm.ntt(dev(x), p))
        assert np.array_equal(X, op.ntt(x, p, g))
        y = host(pm.ntt(dev(X), p, inverse=True))
        assert np.array_equal(y, x)
        assert pm.stream_check() == 0


def test_ntt_hook_large_sampled(gpu_lib):
    """The hooks' four-step plans at 2^22 and 2^23 (rows of 2^13) and 2^24
    (rows of 2^14, columns of at most 2^10): natural-order outputs sampled
    against evaluation at w^k, and the inverse round trip compared whole."""
    pm = gpu_lib
    for p, g, logn in ((2013265921, 31, 22), (998244353, 3, 23), (2013265921, 31, 24)):
        n = 1 << logn
        say("case: ntt large", p, n)
        x = inputs.uniform_mod(inputs.rng_for((105, logn)), n, p)
        X = pm.ntt(dev(x), p)
        Xh = host(X)
        w = op.root(p, g, n)
        for k in (0, 1, n // 2 - 1, n // 2, n - 1):
            assert int(Xh[k]) == op.eval_at(x, p, pow(w, k, p)), (p, n, k)
        y = host(pm.ntt(X, p, inverse=True))
        assert np.array_equal(y, x)
        assert pm.stream_check() == 0
        del X


@pytest.mark.parametrize("p,g", PRIMES[:2])
def test_tft_and_itft_hooks(gpu_lib, p, g):
    pm = gpu_lib
    for logL in (1, 3, 5, 6, 9, 12, 14, 15, 17):
        L = 1 << logL
        gran = pm.itft_granularity(L)
        for z in sorted({1, max(1, L // 3), L}):
            for n in sorted({1, max(1, L // 2 + 1), L - 1 if L > 1 else 1, L}):
                say("case: tft", p, L, z, n)
                x = inputs.uniform_mod(inputs.rng_for((103, logL, z, n)), z, p)
                got = host(pm.tft(dev(x), L, n, p))
                assert np.array_equal(got, op.tft(x, z, L, n, p, g)), (L, z, n)
        # ITFT: values of u (deg < n) at the first n bit-reversed points -> L u
        for n in sorted({gran, L // 2 if L >= 2 * gran else gran, L - gran if L > gran else gran, L}):
            if n % gran or n < 1:
                continue
            say("case: itft", p, L, n)
            u = inputs.uniform_mod(inputs.rng_for((104, logL, n)), n, p)
            v = op.tft(u, n, L, n, p, g)
            got = host(pm.itft(dev(v), L, p))
            want = (u.astype(np.uint64) * (L % p) % p).astype(np.uint32)
            assert np.array_equal(got, want), (L, n)


def test_int_mul(gpu_lib):
    pm = gpu_lib
    rng = np.random.default_rng(9)
    for na, nb in ((1, 1), (2, 3), (64, 64), (1000, 999), (3000, 5000), (70000, 65537), (100001, 77777),
                   (1 << 17, 1 << 17)):
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        want = op.int_mul(a, b)
        for digits in (None, 16):
            say("case: int", na, nb, "digits", digits)
            got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=digits))
            assert np.array_equal(got, want), (na, nb, digits)
    # all-0xFFFF limbs: the longest carry chains
    for n in (100, 5000, 1 << 16, 100001):
        for digits in (None, 16):
            say("case: int ffff", n, "digits", digits)
            ff = np.full(n, 0xFFFF, dtype=np.uint16)
            got = host(pm.int_mul(dev(ff, np.uint16), dev(ff, np.uint16), digits=digits))
            assert np.array_equal(got, op.int_mul(ff, ff)), (n, digits)
    # a product of 0xFFFF..FF by 1 is one propagate chain across every run of
    # limbs (carry maps of the identity), and an output that is not 16-byte
    # aligned takes the limb-by-limb stores
    import torch

    for n in (1, 4095, 4096, 4097, 20000, 140001, 140002):
        say("case: int chain and unaligned output", n)
        ff = np.full(n, 0xFFFF, dtype=np.uint16)
        one = np.ones(1, dtype=np.uint16)
        buf = torch.full((n + 2,), 0x5A5A, dtype=torch.int32).to(torch.uint16).cuda()
        out = buf[1:n + 2]  # n + 1 limbs at an offset of 2 bytes
        pm.int_mul(dev(ff, np.uint16), dev(one, np.uint16), out=out)
        assert pm.stream_check() == 0
        h = host(buf)
        assert np.array_equal(h[1:], op.int_mul(ff, one)) and h[0] == 0x5A5A, n


def test_int_mul_digits32(gpu_lib):
    """32-bit digits (pairs of limbs): forced where the plans allow it,
    refused where they do not, exact against CPython with odd and even limb
    counts, operands of very different lengths, carry runs that span many
    work-groups (0xFFFF..FF times a one-limb integer: every run propagates)
    and an output that is not 16-byte aligned."""
    import torch

    pm = gpu_lib
    rng = np.random.default_rng(91)
    for na, nb in ((70000, 65537), (100001, 77777), (65536, 65535), (300001, 2000), (1 << 18, 1 << 18)):
        say("case: int digits 32", na, nb)
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=32))
        assert pm.stream_check() == 0
        assert np.array_equal(got, op.int_mul(a, b)), (na, nb)
    for n in (200001, 200002):
        for m, fill in ((1, 1), (3, 0xFFFF)):
            say("case: int digits 32 chain, unaligned output", n, m)
            ff = np.full(n, 0xFFFF, dtype=np.uint16)
            y = np.full(m, fill, dtype=np.uint16)
            buf = torch.full((n + m + 1,), 0x5A5A, dtype=torch.int32).to(torch.uint16).cuda()
            out = buf[1:]
            pm.int_mul(dev(ff, np.uint16), dev(y, np.uint16), out=out, digits=32)
            assert pm.stream_check() == 0
            h = host(buf)
            assert np.array_equal(h[1:], op.int_mul(ff, y)) and h[0] == 0x5A5A, (n, m)
    # operands that are not 4-byte aligned: the limb pairs are loaded one limb at a time
    for na, nb in ((90001, 80000), (80000, 90001)):
        say("case: int digits 32, operands at odd limb offsets", na, nb)
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        ta = torch.from_numpy(np.concatenate([[7], a]).astype(np.uint16)).cuda()[1:]
        tb = torch.from_numpy(np.concatenate([[7], b]).astype(np.uint16)).cuda()[1:]
        assert ta.data_ptr() % 4 == 2 and tb.data_ptr() % 4 == 2
        got = host(pm.int_mul(ta, tb, digits=32))
        assert pm.stream_check() == 0
        assert np.array_equal(got, op.int_mul(a, b)), (na, nb)
    # too short for a shared four-step plan at the digit length: refused
    a = rng.integers(0, 1 << 16, 1000, dtype=np.uint16)
    with pytest.raises(pm.PolymulError) as e:
        pm.int_mul(dev(a, np.uint16), dev(a, np.uint16), digits=32)
    assert e.value.status == 2  # PM_EUNSUPPORTED
    with pytest.raises(pm.PolymulError) as e:
        pm.int_mul(dev(a, np.uint16), dev(a, np.uint16), digits=24)
    assert e.value.status == 1  # PM_EINVAL


def test_int_mul_plans_differ(gpu_lib):
    """With one plan for the three primes, each pass runs once over the three
    products; with plans that differ (one pinned here) the products run one
    after the other (16-bit digits), and 32-bit digits are refused.  Both
    give the exact product."""
    pm = gpu_lib
    rng = np.random.default_rng(19)
    primes = (469762049, 998244353, 167772161)
    for digits, (na, nb) in ((16, (40000, 39000)), (32, (80000, 77999))):
        lc = na + nb - 1 if digits == 16 else (na + 1) // 2 + (nb + 1) // 2 - 1
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        want = op.int_mul(a, b)
        base = pm.plan_for(lc, primes[0])
        assert base.kind == 2 and all(pm.plan_for(lc, p).as_tuple() == base.as_tuple() for p in primes)
        t = list(base.as_tuple())
        t[7] = t[7] + 1 if t[4] - t[7] > 3 else t[7] - 1  # twice or half the row threads
        try:
            for pinned in (None, pm.Plan(*t)):
                say("case: int plans", digits, pinned.as_tuple() if pinned else "shared")
                if pinned:
                    pm.plan_cache_put(lc, primes[1], pinned)
                if pinned and digits == 32:
                    with pytest.raises(pm.PolymulError):
                        pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=32)
                    got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16)))  # falls back to 16-bit digits
                else:
                    got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=digits))
                assert pm.stream_check() == 0
                assert np.array_equal(got, want), (digits, pinned)
        finally:
            pm.plan_cache_clear()


def test_int_mul_three_prime_column_passes(gpu_lib):
    """The fused three-prime column passes (first radix 16, 2^2 .. 2^5 second
    radix, pinned for all three primes so the passes are shared): exact
    against CPython, including all-0xFFFF operands (the longest carry chains)
    and lengths that end mid-tile."""
    pm = gpu_lib
    rng = np.random.default_rng(29)
    primes = (469762049, 998244353, 167772161)
    try:
        for log_rb, log_c, (n1, n2) in ((2, 10, (40000, 25537)), (3, 10, (70001, 60000)), (4, 10, (131072, 100000)),
                                        (5, 10, (200000, 262144))):
            # 16-bit digits: na, nb limbs; 32-bit digits: the same digit
            # counts from 2 n1 - 1 (odd) and 2 n2 limbs
            for digits, (na, nb) in ((16, (n1, n2)), (32, (2 * n1 - 1, 2 * n2))):
                lc = n1 + n2 - 1
                log_l = (lc - 1).bit_length()
                assert log_l == 4 + log_rb + log_c
                gran = 1 << (log_l - 4)
                plan = pm.Plan(2, log_l, 4, log_rb, log_c, (lc + gran - 1) // gran, 3, log_c - 4)
                pm.plan_cache_clear()
                for p in primes:
                    pm.plan_cache_put(lc, p, plan)
                for ff in (False, True):
                    say("case: int fused", digits, plan.as_tuple(), na, nb, "ffff" if ff else "random")
                    if ff:
                        a = np.full(na, 0xFFFF, dtype=np.uint16)
                        b = np.full(nb, 0xFFFF, dtype=np.uint16)
                    else:
                        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
                        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
                    got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=digits))
                    assert pm.stream_check() == 0
                    assert np.array_equal(got, op.int_mul(a, b)), (digits, plan.as_tuple(), ff)
    finally:
        pm.plan_cache_clear()


def test_int_mul_first_radix_32(gpu_lib):
    """The fused three-prime passes with the first radix 32 (a lane pair per
    inverse task) for 29 .. 32 kept blocks and second radices 2^2 .. 2^5, and
    a plan of first radix 32 with 20 kept blocks, which the integer product
    runs as its radix-16 twin: exact against CPython."""
    pm = gpu_lib
    rng = np.random.default_rng(31)
    primes = (469762049, 998244353, 167772161)
    cases = ((2, 10, 29, (60000, 57000), True), (3, 10, 30, (130000, 110000), False),
             (4, 10, 31, (260000, 240000), False), (5, 10, 32, (524288, 500000), True),
             (5, 11, 20, (700000, 600000), False))
    try:
        for log_rb, log_c, ma, (n1, n2), ff in cases:
            for digits, (na, nb) in ((16, (n1, n2)), (32, (2 * n1, 2 * n2 - 1))):
                lc = n1 + n2 - 1
                log_l = 5 + log_rb + log_c
                gran = 1 << (log_l - 5)
                assert (lc - 1).bit_length() == log_l and (lc + gran - 1) // gran == ma
                plan = pm.Plan(2, log_l, 5, log_rb, log_c, ma, 3, log_c - 4)
                pm.plan_cache_clear()
                for p in primes:
                    pm.plan_cache_put(lc, p, plan)
                for f in ((False, True) if ff else (False,)):
                    say("case: int fused radix 32", digits, plan.as_tuple(), na, nb, "ffff" if f else "random")
                    if f:
                        a = np.full(na, 0xFFFF, dtype=np.uint16)
                        b = np.full(nb, 0xFFFF, dtype=np.uint16)
                    else:
                        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
                        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
                    got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=digits))
                    assert pm.stream_check() == 0
                    assert np.array_equal(got, op.int_mul(a, b)), (digits, plan.as_tuple(), f)
    finally:
        pm.plan_cache_clear()


def test_int_mul_full_size(gpu_lib):
    """Two random 2^21-limb integers, bit-exact against CPython's multiply,
    with 32-bit digits (2^21-point transforms) and 16-bit digits (2^22)."""
    pm = gpu_lib
    a, b = inputs.int_operands()
    want = op.int_mul(a, b)
    for digits in (None, 16):
        say("case: int 2^21 x 2^21, digits", digits)
        got = host(pm.int_mul(dev(a, np.uint16), dev(b, np.uint16), digits=digits))
        assert pm.stream_check() == 0
        assert np.array_equal(got, want), digits


def test_batch_matches_oracle(gpu_lib):
    """Uneven lengths, mixed primes, one graph launch; the second call with the
    same shape replays the cached graph with new data."""
    pm = gpu_lib
    for rep, tag in enumerate(((105,), (106,))):
        items = inputs.batch_uneven(count=96, lo=1, hi=20000, tag=tag)
        # same shape both times: reuse the first draw's lengths and primes
        if rep == 1:
            rng = np.random.default_rng(3)
            items = [inputs.BatchItem(rng.integers(0, it.p, it.a.size, dtype=np.uint32),
                                      rng.integers(0, it.p, it.b.size, dtype=np.uint32), it.p) for it in first]
        first = items
        say("case: batch 96 rep", rep)
        outs = pm.poly_mul_batch([(dev(it.a), dev(it.b), it.p) for it in items])
        assert pm.stream_check() == 0
        for it, c in zip(items, outs):
            assert np.array_equal(host(c), op.poly_mul(it.a, it.b, it.p))


def test_batch_one_work_group_lengths_share_a_launch(gpu_lib):
    """The batch's one-work-group products of 2^6 .. 2^11 points (default
    plans, first radix 8) run as one launch per value range of the prime,
    whatever their lengths: under tracing (the classes one after the other)
    a batch with lengths from 65 to 2047 outputs over all four primes makes
    exactly two such launches, and every product is exact."""
    pm = gpu_lib
    items = inputs.batch_uneven(count=200, lo=33, hi=1024, tag=(118,))
    lcs = [it.a.size + it.b.size - 1 for it in items]
    assert min(lcs) > 64 and max(lcs) <= 2047
    assert len({it.p for it in items}) == 4
    pm.plan_cache_clear()
    for lc, it in zip(lcs, items):
        P = pm.plan_for(lc, it.p)
        assert P.kind == 1 and P.log_ra == 3 and P.log_l <= 11, (lc, P)
    probs = [(dev(it.a), dev(it.b), it.p) for it in items]
    say("case: batch of one-work-group lengths 65..2047")
    pm.trace_reset()
    pm.trace_enable(True)
    try:
        outs = pm.poly_mul_batch(probs)
        assert pm.stream_check() == 0
    finally:
        pm.trace_enable(False)
    tot, n = pm.trace_query("lds_conv")
    pm.trace_reset()
    assert n == 2, n
    for it, c in zip(items, outs):
        assert np.array_equal(host(c), op.poly_mul(it.a, it.b, it.p))
    # and in the captured graph (tracing off), the same products again
    outs = pm.poly_mul_batch(probs)
    assert pm.stream_check() == 0
    for it, c in zip(items, outs):
        assert np.array_equal(host(c), op.poly_mul(it.a, it.b, it.p))


def test_batch_uneven_4096(gpu_lib):
    """The full batch: 4096 products, lengths log-uniform in [64, 65536], four
    primes; every product against the oracle's transform route, and sampled
    coefficients against the defining sum."""
    pm = gpu_lib
    items = inputs.batch_uneven()
    say("case: batch 4096")
    outs = pm.poly_mul_batch([(dev(it.a), dev(it.b), it.p) for it in items])
    assert pm.stream_check() == 0
    rng = np.random.default_rng(4)
    for k, (it, c) in enumerate(zip(items, outs)):
        got = host(c)
        assert np.array_equal(got, op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p])), k
        if k % 64 == 0:
            ks = rng.integers(0, got.size, 8)
            assert np.array_equal(got[ks], op.poly_mul_sample(it.a, it.b, it.p, ks))


@pytest.mark.parametrize("p,g", PRIMES)
def test_cyclic_and_negacyclic_products(gpu_lib, p, g):
    """Products mod x^n - 1 and x^n + 1 (eq. 5 and the factors of eq. 13) for the
    defining-sum, one-work-group and four-step plans, operands shorter than n
    included: against the linear product reduced mod x^n -+ 1, and for small n
    against the oracle's defining sums directly."""
    pm = gpu_lib
    cases = ((4, 4, 3), (64, 64, 30), (128, 128, 128), (2048, 1000, 2048), (16384, 16384, 16384),
             (32768, 32768, 20000), (1 << 17, 1 << 17, 1 << 17), (1 << 20, 1 << 20, 777777))
    for k, (n, la, lb) in enumerate(cases):
        say("case:", p, n, la, lb)
        a, b = inputs.poly_pair((150, k, p % 1000), la, lb, p)
        lin = op.poly_mul(a, b, p) if la * lb <= 1 << 24 else op.poly_mul_ntt(a, b, p, g)
        got_c = host(pm.cyclic_mul(dev(a), dev(b), n, p))
        got_n = host(pm.negacyclic_mul(dev(a), dev(b), n, p))
        assert pm.stream_check() == 0
        assert np.array_equal(got_c, op.fold(lin, n, p, +1)), ("cyclic", n)
        assert np.array_equal(got_n, op.fold(lin, n, p, -1)), ("negacyclic", n)
        if n <= 2048:
            ap = np.zeros(n, np.uint32)
            bp = np.zeros(n, np.uint32)
            ap[:la], bp[:lb] = a, b
            assert np.array_equal(got_c, op.cyclic_conv(ap, bp, p))
            assert np.array_equal(got_n, op.negacyclic_conv(ap, bp, p))


# odd factors q of p - 1 with kernels for the prime-factor split
MIXED_Q = {2013265921: (3, 5, 15), 998244353: (7, 17), 469762049: (7,), 167772161: (5,)}


@pytest.mark.parametrize("p,g", PRIMES)
def test_mixed_length_ntt(gpu_lib, p, g):
    """Transforms of length n = q 2^k (q odd, q | p - 1) by the prime-factor
    split: every output against the evaluation definition up to n = 8192,
    sampled outputs (first, last and 64 random) beyond; the inverse against
    the same definition and the exact round trip."""
    pm = gpu_lib
    for q in MIXED_Q[p]:
        for k in (0, 1, 3, 6, 9, 12, 15, 17):
            n = q << k
            say("case: mixed ntt", p, q, n)
            x = inputs.uniform_mod(inputs.rng_for((160, q, k, p % 1000)), n, p)
            X = host(pm.ntt(dev(x), p))
            Y = host(pm.ntt(dev(x), p, inverse=True))
            assert pm.stream_check() == 0
            if n <= 8192:
                ks = list(range(n))
            else:
                ks = sorted(set([0, 1, n - 1] + random.Random(n).sample(range(n), 64)))
            assert np.array_equal(X[ks], op.dft_eval(x, p, g, ks=ks)), (q, n)
            assert np.array_equal(Y[ks], op.dft_eval(x, p, g, inverse=True, ks=ks)), (q, n)
            assert np.array_equal(host(pm.ntt(dev(X), p, inverse=True)), x), (q, n)


@pytest.mark.parametrize("p,g", PRIMES)
def test_mixed_radix_products(gpu_lib, p, g):
    """Products through circular convolutions of length q 2^k >= la + lb - 1:
    rows by the defining sums (2^k <= 64), one work-group and four-step rows,
    ragged lengths; every output against the schoolbook oracle."""
    pm = gpu_lib
    shapes = [(1, 1), (2, 1), (10, 7), (40, 30), (100, 93), (1000, 537), (5000, 4001), (20000, 13001),
              (70000, 30001)]
    for q in MIXED_Q[p]:
        for i, (la, lb) in enumerate(shapes):
            say("case: mixed product", p, q, la, lb)
            a, b = inputs.poly_pair((161, q, i, p % 1000), la, lb, p)
            got = host(pm.poly_mul_mixed(dev(a), dev(b), p, q))
            assert pm.stream_check() == 0
            assert np.array_equal(got, op.poly_mul(a, b, p)), (q, la, lb)


def test_mixed_radix_product_large_sampled(gpu_lib):
    """3 * 2^19 x 3 * 2^19 mod 2013265921 through length 3 * 2^20 (rows of 2^20,
    four-step), and 600001 x 400000 through length 5 * 2^18: 256 sampled outputs
    each against the oracle's defining sum."""
    pm = gpu_lib
    p = 2013265921
    for q, la, lb in ((3, 3 << 19, 3 << 19), (5, 600001, 400000)):
        say("case: mixed product large", q, la, lb)
        a, b = inputs.poly_pair((162, q), la, lb, p)
        got = host(pm.poly_mul_mixed(dev(a), dev(b), p, q))
        assert pm.stream_check() == 0
        rng = random.Random(q)
        ks = sorted(set([0, got.size - 1] + rng.sample(range(got.size), 256)))
        assert np.array_equal(got[ks], op.poly_mul_sample(a, b, p, ks))


def test_mixed_radix_errors(gpu_lib):
    import ctypes

    pm = gpu_lib
    x = dev(np.ones(100, np.uint32))
    for p, q in ((998244353, 3), (2013265921, 7), (2013265921, 9), (167772161, 1)):
        with pytest.raises(pm.PolymulError) as e:
            pm.poly_mul_mixed(x, x, p, q)
        assert e.value.status == pm.PM_EUNSUPPORTED, (p, q)
    with pytest.raises(pm.PolymulError) as e:
        pm.ntt(dev(np.ones(18, np.uint32)), 2013265921)  # odd part 9
    assert e.value.status == pm.PM_EUNSUPPORTED
    # 3 * 2^25: the power-of-two part is beyond 2^24; rejected before any launch
    st = pm.lib().pm_ntt(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 3 << 25, 2013265921, 0, None)
    assert st == pm.PM_ETOOLARGE
    a = np.full(3000, 5, dtype=np.uint32)
    a[1234] = 2013265921  # not canonical
    pm.poly_mul_mixed(dev(a), x, 2013265921, 3)
    assert pm.stream_check() == pm.PM_ENOTREDUCED
    assert pm.stream_check() == 0


def test_general_radix_plan_pinned(gpu_lib):
    """A pinned general-radix plan (kind 3: the product through length
    5 * 2^13 = 40960 for 40000 outputs) drives products alone, while a batch
    and the allocation-free entry point, which run power-of-two plans only,
    take their own plans; every result against the schoolbook oracle."""
    import torch

    pm = gpu_lib
    p = 2013265921
    la, lb = 25001, 15000
    lc = la + lb - 1
    P = [Q for Q in pm.plan_candidates(lc, p) if Q.kind == pm.PLAN_MIXED and Q.q == 5][0]
    assert P.log_l == 13
    a, b = inputs.poly_pair((170, lc), la, lb, p)
    want = op.poly_mul(a, b, p)
    pm.plan_cache_clear()
    try:
        pm.plan_cache_put(lc, p, P)
        assert pm.plan_for(lc, p).as_tuple() == P.as_tuple()
        assert pm.plan_for(lc, p, context=pm.CTX_BATCH).kind != pm.PLAN_MIXED
        say("case: pinned general radix alone", P)
        assert np.array_equal(_product(pm, a, b, p), want)
        say("case: pinned general radix in a batch")
        outs = pm.poly_mul_batch([(dev(a), dev(b), p), (dev(b), dev(a), p)])
        assert pm.stream_check() == 0
        assert all(u.kind != pm.PLAN_MIXED for u in pm.batch_plans_used(2))
        for o in outs:
            assert np.array_equal(host(o), want)
        say("case: pinned general radix, allocation-free entry point")
        pm.init()
        out = torch.empty(lc, dtype=torch.uint32, device="cuda")
        pm.poly_mul_noalloc(dev(a), dev(b), p, out)
        assert pm.stream_check() == 0
        assert np.array_equal(host(out), want)
    finally:
        pm.plan_cache_clear()


def _eval2(c, p, x, y):
    """c(x, y) mod p for a 2-D coefficient array, vectorised with exact int64 steps."""
    c = np.asarray(c, dtype=np.int64)
    yp = np.array([pow(y, j, p) for j in range(c.shape[1])], dtype=np.int64)
    xp = np.array([pow(x, i, p) for i in range(c.shape[0])], dtype=np.int64)
    rows = ((c * yp[None, :]) % p).sum(axis=1) % p
    return int(((rows * xp) % p).sum() % p)


def test_multivariate_products(gpu_lib):
    """Kronecker substitution: against the multivariate definition on small
    boxes (one to four variables), and a 1024 x 1024 by 1024 x 1024 bivariate
    product (2047^2 coefficients, a 2^22 transform) against evaluation at
    random points."""
    pm = gpu_lib
    rng = np.random.default_rng(160)
    for p in (998244353, 2013265921):
        for k, (sa, sb) in enumerate((((1000,), (777,)), ((30, 40), (25, 17)), ((5, 6, 7), (4, 3, 9)),
                                      ((3, 2, 4, 5), (2, 5, 3, 2)), ((1, 64), (1, 1)), ((40, 1), (1, 33)))):
            say("case: multivariate", p, sa, sb)
            a = rng.integers(0, p, sa, dtype=np.uint32)
            b = rng.integers(0, p, sb, dtype=np.uint32)
            got = host(pm.poly_mul_multi(dev(a), dev(b), p))
            assert pm.stream_check() == 0
            assert np.array_equal(got, op.poly_mul_multi(a, b, p)), (sa, sb)
    p = 2013265921
    say("case: multivariate 1024^2 x 1024^2")
    a = rng.integers(0, p, (1024, 1024), dtype=np.uint32)
    b = rng.integers(0, p, (1024, 1024), dtype=np.uint32)
    got = host(pm.poly_mul_multi(dev(a), dev(b), p))
    assert got.shape == (2047, 2047) and pm.stream_check() == 0
    for _ in range(4):
        x, y = (int(t) for t in rng.integers(1, p, 2))
        assert _eval2(got, p, x, y) == _eval2(a, p, x, y) * _eval2(b, p, x, y) % p
    # one row of the result by the definition: c[i, :] = sum_r a[r, :] * b[i - r, :]
    i = 700
    row = np.zeros(2047, dtype=np.int64)
    for r in range(max(0, i - 1023), min(i, 1023) + 1):
        row = (row + op.poly_mul(a[r], b[i - r], p).astype(np.int64)) % p
    assert np.array_equal(got[i], row.astype(np.uint32))


def test_ring_product_errors(gpu_lib):
    pm = gpu_lib
    p = 998244353
    x = dev(np.ones(100, np.uint32))
    for fn in (pm.cyclic_mul, pm.negacyclic_mul):
        with pytest.raises(pm.PolymulError) as e:
            fn(x, x, 96, p)  # not a power of two
        assert e.value.status == pm.PM_EINVAL
        with pytest.raises(pm.PolymulError) as e:
            fn(x, x, 64, p)  # operands longer than n
        assert e.value.status == pm.PM_EINVAL
    with pytest.raises(pm.PolymulError) as e:
        pm.negacyclic_mul(x, x, 1 << 23, p)  # 2n does not divide p - 1
    assert e.value.status == pm.PM_ETOOLARGE


def test_products_on_concurrent_streams(gpu_lib):
    """Products and batches issued on two streams without synchronising
    between them: each stream has its own workspace, so every result is exact."""
    import torch

    pm = gpu_lib
    p = 2013265921
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    pairs = [inputs.poly_pair((130, k), la, lb, p) for k, (la, lb) in enumerate(((300000, 200001), (150000, 150000),
                                                                                  (70001, 9000), (4096, 4096)))]
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    items = inputs.batch_uneven(count=64, lo=1, hi=30000, tag=(131,))
    ditems = [(dev(it.a), dev(it.b), it.p) for it in items]
    torch.cuda.synchronize()
    say("case: two streams, 4 products x 3 rounds + one batch each")
    outs = []
    for rnd in range(3):
        for k, (da, db) in enumerate(dpairs):
            s = s1 if (k + rnd) % 2 == 0 else s2
            with torch.cuda.stream(s):
                outs.append((k, pm.poly_mul(da, db, p, stream=s)))
    b1 = pm.poly_mul_batch(ditems[:32], stream=s1)
    b2 = pm.poly_mul_batch(ditems[32:], stream=s2)
    torch.cuda.synchronize()
    assert pm.stream_check() == 0
    for k, c in outs:
        a, b = pairs[k]
        assert np.array_equal(host(c), op.poly_mul_ntt(a, b, p, inputs.PRIMES[p])), k
    for it, c in zip(items, b1 + b2):
        assert np.array_equal(host(c), op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p]))


def test_caller_owned_workspace(gpu_lib):
    """Products, an integer product and a batch on a stream whose workspace
    the caller supplied (sized by the queries): exact results; a workspace
    that is too small is refused with PM_ENOMEM before anything runs, and the
    stream returns to the library's own workspace afterwards."""
    import torch

    pm = gpu_lib
    p = 2013265921
    s = torch.cuda.Stream()
    pairs = [inputs.poly_pair((170, k), la, lb, p) for k, (la, lb) in enumerate(((600001, 400000), (1 << 20, 1 << 20),
                                                                                  (70001, 9000), (1000, 999)))]
    ia, ib = inputs.int_operands(1 << 12, tag=171)
    items = inputs.batch_uneven(count=40, lo=1, hi=40000, tag=(172,))
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    ditems = [(dev(it.a), dev(it.b), it.p) for it in items]
    need = max([pm.workspace_query(a.size, b.size, p) for a, b in pairs] +
               [pm.int_mul_workspace_query(ia.size, ib.size), pm.batch_workspace_query(ditems)])
    say("case: caller workspace of", need, "bytes")
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    pm.set_workspace(buf, stream=s)
    try:
        with torch.cuda.stream(s):
            outs = [pm.poly_mul(da, db, p, stream=s) for da, db in dpairs]
            ic = pm.int_mul(dev(ia, np.uint16), dev(ib, np.uint16), stream=s)
            bouts = pm.poly_mul_batch(ditems, stream=s)
        s.synchronize()
        assert pm.stream_check() == 0
        for (a, b), c in zip(pairs, outs):
            assert np.array_equal(host(c), op.poly_mul_ntt(a, b, p, inputs.PRIMES[p]))
        assert np.array_equal(host(ic), op.int_mul(ia, ib))
        for it, c in zip(items, bouts):
            assert np.array_equal(host(c), op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p]))
        # too small for the 2^20 x 2^20 product: refused, nothing written
        small = pm.workspace_query(1 << 20, 1 << 20, p) - 4096
        pm.set_workspace(buf[:small], stream=s)
        da, db = dpairs[1]
        sentinel = torch.full((da.numel() + db.numel() - 1,), 7, dtype=torch.uint32, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(pm.PolymulError) as e:
            pm.poly_mul(da, db, p, out=sentinel, stream=s)
        assert e.value.status == pm.PM_ENOMEM
        s.synchronize()
        assert bool((sentinel == 7).all())
    finally:
        pm.set_workspace(None, stream=s)
    with torch.cuda.stream(s):
        c = pm.poly_mul(*dpairs[1], p, stream=s)
    s.synchronize()
    a, b = pairs[1]
    assert np.array_equal(host(c), op.poly_mul_ntt(a, b, p, inputs.PRIMES[p]))


def test_integer_product_workspace_is_exact(gpu_lib):
    """Under the default policy the integer product's workspace query is the
    exact need of the layout the call takes (32-bit digits here, and 16-bit
    ones when forced): a caller workspace of that size runs the product
    exactly; 256 bytes less is refused with PM_ENOMEM and nothing is
    written."""
    import torch

    pm = gpu_lib
    rng = np.random.default_rng(173)
    na, nb = 100001, 77777
    a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
    b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
    want = op.int_mul(a, b)
    ta, tb = dev(a, np.uint16), dev(b, np.uint16)
    s = torch.cuda.Stream()
    pm.plan_cache_clear()
    try:
        for digits in (None, 16):
            need = pm.int_mul_workspace_query(na, nb, digits=digits)
            say("case: integer product in an exact workspace", digits, need)
            buf = torch.empty(need, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            pm.set_workspace(buf, stream=s)
            with torch.cuda.stream(s):
                c = pm.int_mul(ta, tb, stream=s, digits=digits)
            s.synchronize()
            assert pm.stream_check() == 0
            assert np.array_equal(host(c), want), digits
            pm.set_workspace(buf[:need - 256], stream=s)
            out = torch.full((na + nb,), 0x5A5A, dtype=torch.int32).to(torch.uint16).cuda()
            torch.cuda.synchronize()
            with pytest.raises(pm.PolymulError) as e:
                pm.int_mul(ta, tb, out=out, stream=s, digits=digits)
            assert e.value.status == pm.PM_ENOMEM
            s.synchronize()
            assert bool((out == 0x5A5A).all())
            pm.set_workspace(None, stream=s)
    finally:
        pm.set_workspace(None, stream=s)


def test_not_reduced_input_is_reported(gpu_lib):
    pm = gpu_lib
    p = 998244353
    for la in (10, 3000, 40000):
        a = np.full(la, 5, dtype=np.uint32)
        a[la // 2] = p  # not canonical
        b = np.ones(7, dtype=np.uint32)
        say("case: not reduced", la)
        pm.poly_mul(dev(a), dev(b), p)
        assert pm.stream_check() == pm.PM_ENOTREDUCED
        assert pm.stream_check() == 0  # cleared


def test_host_errors_raise(gpu_lib):
    pm = gpu_lib
    a = dev(np.ones(8))
    with pytest.raises(pm.PolymulError) as e:
        pm.poly_mul(a, a, 1000000007)
    assert e.value.status == pm.PM_EUNSUPPORTED
