"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's own formula: each checks it against a
different route to the same value (hand-worked fixtures, closed forms,
Kronecker substitution through CPython's big integers, evaluation at random
points, the convolution theorem, a second algorithm).  The last group plants
plausible mistakes in copies of the oracle and shows that a pin catches each.
"""

import math
import random

import numpy as np
import pytest

from conftest import golden
from oracle import mlp as omlp
from oracle import poly as op
from paper_1609_01010_amd import inputs

PRIMES = list(inputs.PRIMES.items())


def _records(name):
    recs = golden(name)
    out = []
    cur = {}
    for k, v in recs:
        if k in cur:
            out.append(cur)
            cur = {}
        cur[k] = v
    out.append(cur)
    return out


# --- product pins -------------------------------------------------------------

def kronecker_product(a, b, p):
    """a*b mod p through one CPython integer multiply (Kronecker substitution):
    pack the coefficients 96 bits apart, multiply, unpack, reduce."""
    S = 96
    A = sum(int(x) << (S * i) for i, x in enumerate(a))
    B = sum(int(x) << (S * i) for i, x in enumerate(b))
    C = A * B
    mask = (1 << S) - 1
    return [((C >> (S * k)) & mask) % p for k in range(len(a) + len(b) - 1)]


def check_product(mul):
    """Pins of a product routine mul(a, b, p) -> coefficients."""
    # hand-worked fixtures (Def. 2, eq. 2)
    for rec in _records("product_small.txt"):
        got = [int(x) for x in mul(rec["a"], rec["b"], rec["p"][0])]
        assert got == rec["c"]
    rng = random.Random(1)
    for p, _ in PRIMES[:2]:
        # brute force on all small shapes, random and extreme values
        for la in range(1, 7):
            for lb in range(1, 7):
                for vals in ("rand", "max", "mixed"):
                    if vals == "rand":
                        a = [rng.randrange(p) for _ in range(la)]
                        b = [rng.randrange(p) for _ in range(lb)]
                    elif vals == "max":
                        a = [p - 1] * la
                        b = [p - 1] * lb
                    else:
                        a = [rng.choice([0, 1, p - 1]) for _ in range(la)]
                        b = [rng.choice([0, 1, p - 1]) for _ in range(lb)]
                    assert [int(x) for x in mul(a, b, p)] == kronecker_product(a, b, p)
        # closed forms: (1+x)^m (1+x)^n = (1+x)^(m+n)
        m, n = 37, 29
        a = [math.comb(m, i) % p for i in range(m + 1)]
        b = [math.comb(n, i) % p for i in range(n + 1)]
        assert [int(x) for x in mul(a, b, p)] == [math.comb(m + n, k) % p for k in range(m + n + 1)]
        # all ones: c_k = number of (i, j) with i + j = k
        la, lb = 13, 8
        got = [int(x) for x in mul([1] * la, [1] * lb, p)]
        assert got == [min(k + 1, la, lb, la + lb - 1 - k) for k in range(la + lb - 1)]
        # geometric: (sum r^i x^i)(sum r^j x^j) -> c_k = #pairs * r^k
        r = 12345
        a = [pow(r, i, p) for i in range(la)]
        b = [pow(r, j, p) for j in range(lb)]
        got = [int(x) for x in mul(a, b, p)]
        assert got == [min(k + 1, la, lb, la + lb - 1 - k) * pow(r, k, p) % p for k in range(la + lb - 1)]
        # monomials: x^i * x^j = x^(i+j)
        a = [0] * 5 + [1]
        b = [0] * 3 + [1]
        got = [int(x) for x in mul(a, b, p)]
        assert got == [0] * 8 + [1]
        # random points: c(x) = a(x) b(x)
        a = [rng.randrange(p) for _ in range(300)]
        b = [rng.randrange(p) for _ in range(211)]
        c = [int(x) for x in mul(a, b, p)]
        for _ in range(8):
            x = rng.randrange(p)
            assert op.eval_at_py(c, p, x) == op.eval_at_py(a, p, x) * op.eval_at_py(b, p, x) % p
        # commutativity
        assert [int(x) for x in mul(b, a, p)] == c


def test_product_schoolbook_pins():
    check_product(op.poly_mul)


def test_product_python_pins():
    check_product(op.poly_mul_py)


def test_product_ntt_route_pins():
    check_product(lambda a, b, p: op.poly_mul_ntt(a, b, p, inputs.PRIMES[p]))


@pytest.mark.parametrize("p,g", PRIMES)
def test_product_routes_agree_medium(p, g):
    a, b = inputs.poly_pair((90, p % 1000), 3001, 1777, p)
    c = op.poly_mul(a, b, p)
    assert np.array_equal(c, op.poly_mul_ntt(a, b, p, g))
    ks = np.array([0, 1, 2, 1776, 1777, 3000, 3001, c.size - 2, c.size - 1])
    assert np.array_equal(op.poly_mul_sample(a, b, p, ks), c[ks])
    rng = random.Random(p)
    for _ in range(4):
        x = rng.randrange(p)
        assert op.eval_at(c, p, x) == op.eval_at(a, p, x) * op.eval_at(b, p, x) % p


def test_random_point_evaluation_large():
    """At the large size only evaluation and a few sampled sums are affordable."""
    p, g = 2013265921, 31
    a, b = inputs.poly_pair((91, 1), 1 << 16, (1 << 16) - 5, p)
    c = op.poly_mul_ntt(a, b, p, g)
    rng = random.Random(7)
    for _ in range(8):
        x = rng.randrange(p)
        assert op.eval_at(c, p, x) == op.eval_at(a, p, x) * op.eval_at(b, p, x) % p
    ks = np.array(sorted(rng.sample(range(c.size), 64)))
    assert np.array_equal(op.poly_mul_sample(a, b, p, ks), c[ks])


# --- transform pins -----------------------------------------------------------

def check_ntt(ntt):
    """Pins of ntt(x, p, g, inverse) -> natural-order transform."""
    rec = _records("transform_p17.txt")[0]
    p, g = rec["p"][0], rec["g"][0]
    assert [int(v) for v in ntt(rec["ntt_in"], p, g, False)] == rec["ntt_out"]
    for p, g in PRIMES:
        for n in (1, 2, 4, 8, 64):
            w = op.root(p, g, n)
            assert pow(w, n, p) == 1
            if n > 1:
                assert pow(w, n // 2, p) == p - 1
            # delta_0 -> all ones, delta_1 -> powers of w
            d0 = [1] + [0] * (n - 1)
            assert [int(v) for v in ntt(d0, p, g, False)] == [1] * n
            if n > 1:
                d1 = [0, 1] + [0] * (n - 2)
                assert [int(v) for v in ntt(d1, p, g, False)] == [pow(w, k, p) for k in range(n)]
        rng = random.Random(p)
        x = [rng.randrange(p) for _ in range(32)]
        assert [int(v) for v in ntt(x, p, g, False)] == op.dft_direct(x, p, g)
        assert [int(v) for v in ntt(x, p, g, True)] == op.dft_direct(x, p, g, inverse=True)
        assert [int(v) for v in ntt(ntt(x, p, g, False), p, g, True)] == x
        # convolution theorem, eq. 8: DFT(u (*) v) = DFT(u) . DFT(v)
        u = [rng.randrange(p) for _ in range(16)]
        v = [rng.randrange(p) for _ in range(16)]
        cyc = [int(t) for t in op.cyclic_conv(u, v, p)]
        lhs = [int(t) for t in ntt(cyc, p, g, False)]
        fu = ntt(u, p, g, False)
        fv = ntt(v, p, g, False)
        assert lhs == [int(s) * int(t) % p for s, t in zip(fu, fv)]


def test_ntt_pins():
    check_ntt(op.ntt)


def test_dft_direct_is_evaluation():
    p, g = 998244353, 3
    x = [5, 7, 11, 13, 17, 19, 23, 29]
    w = op.root(p, g, 8)
    assert op.dft_direct(x, p, g) == [op.eval_at_py(x, p, pow(w, k, p)) for k in range(8)]


# lengths N = q 2^k with q an odd factor of p - 1, per prime
MIXED_LENGTHS = {2013265921: (3, 6, 10, 12, 15, 20, 24, 30, 48, 96),
                 998244353: (7, 14, 17, 28, 34, 56, 68, 112),
                 469762049: (7, 14, 28, 56),
                 167772161: (5, 10, 20, 40, 80)}


def _prime_factors(n):
    f, d = set(), 2
    while d * d <= n:
        while n % d == 0:
            f.add(d)
            n //= d
        d += 1
    if n > 1:
        f.add(n)
    return f


def check_dft_any_length(dft):
    """Pins of a transform dft(x, p, g, inverse) of any length N | p - 1."""
    rng = random.Random(11)
    for p, g in PRIMES:
        for n in MIXED_LENGTHS[p]:
            w = op.root(p, g, n)
            # w has order exactly n
            assert pow(w, n, p) == 1 and all(pow(w, n // r, p) != 1 for r in _prime_factors(n))
            # closed forms: delta_0 -> all ones; delta_1 -> w^k; all ones -> n delta_0
            # (the geometric sum over the n-th roots vanishes only for a root of order n)
            d0 = [1] + [0] * (n - 1)
            d1 = [0, 1] + [0] * (n - 2)
            assert [int(v) for v in dft(d0, p, g, False)] == [1] * n
            assert [int(v) for v in dft(d1, p, g, False)] == [pow(w, k, p) for k in range(n)]
            assert [int(v) for v in dft([1] * n, p, g, False)] == [n % p] + [0] * (n - 1)
            # the convolution theorem (eq. 8) with the circular convolution's defining sums
            u = [rng.randrange(p) for _ in range(n)]
            v = [rng.randrange(p) for _ in range(n)]
            fu, fv = dft(u, p, g, False), dft(v, p, g, False)
            lhs = [int(t) for t in dft(op.cyclic_conv(u, v, p), p, g, False)]
            assert lhs == [int(a) * int(b) % p for a, b in zip(fu, fv)]
            # the inverse undoes the transform, factor n^-1 included
            assert [int(t) for t in dft(fu, p, g, True)] == u
        # power-of-two lengths: the radix-2 algorithm
        x = [rng.randrange(p) for _ in range(64)]
        assert [int(t) for t in dft(x, p, g, False)] == [int(t) for t in op.ntt(x, p, g)]


def test_dft_any_length_pins():
    check_dft_any_length(op.dft_eval)


def _dft_root_of_half_order(x, p, g, inverse):
    n = len(x)
    m = n // 2 if n % 2 == 0 else n
    w = op.root(p, g, m, inverse)
    out = [op.eval_at(x, p, pow(w, k, p)) for k in range(n)]
    return [v * pow(n, p - 2, p) % p for v in out] if inverse else out


def _dft_no_scale(x, p, g, inverse):
    y = op.dft_eval(x, p, g, inverse)
    return [int(v) * len(x) % p for v in y] if inverse else y


def _dft_shifted_index(x, p, g, inverse):
    n = len(x)
    w = op.root(p, g, n, inverse)
    out = [op.eval_at(x, p, pow(w, k + 1, p)) for k in range(n)]
    return [v * pow(n, p - 2, p) % p for v in out] if inverse else out


@pytest.mark.parametrize("mutant", [_dft_root_of_half_order, _dft_no_scale, _dft_shifted_index])
def test_dft_any_length_pins_catch_mistakes(mutant):
    with pytest.raises(AssertionError):
        check_dft_any_length(mutant)


def test_cyclic_conv_is_product_mod_xn_minus_1():
    """Def. 4: circular convolution = product reduced mod x^N - 1."""
    p = 469762049
    rng = random.Random(3)
    n = 23
    u = [rng.randrange(p) for _ in range(n)]
    v = [rng.randrange(p) for _ in range(n)]
    full = kronecker_product(u, v, p)
    fold = [0] * n
    for k, c in enumerate(full):
        fold[k % n] = (fold[k % n] + c) % p
    assert [int(t) for t in op.cyclic_conv(u, v, p)] == fold


def test_negacyclic_conv_is_product_mod_xn_plus_1():
    """The nega-circular factor of eq. 13: the product reduced mod x^N + 1
    (x^N = -1), against the product by Kronecker substitution."""
    p = 2013265921
    rng = random.Random(31)
    for n in (1, 2, 7, 23, 64):
        u = [rng.randrange(p) for _ in range(n)]
        v = [rng.randrange(p) for _ in range(n)]
        full = kronecker_product(u, v, p)
        fold = [0] * n
        for k, c in enumerate(full):
            fold[k % n] += c if (k // n) % 2 == 0 else -c
        assert [int(t) for t in op.negacyclic_conv(u, v, p)] == [f % p for f in fold]


def test_negacyclic_closed_forms():
    """x^(N-1) x = x^N = -1 mod x^N + 1 (and +1 mod x^N - 1); x^i x^j = x^(i+j)
    below N in both rings."""
    p, n = 998244353, 16
    u = [0] * n
    v = [0] * n
    u[n - 1], v[1] = 1, 1
    neg = op.negacyclic_conv(u, v, p)
    cyc = op.cyclic_conv(u, v, p)
    assert int(neg[0]) == p - 1 and not neg[1:].any()
    assert int(cyc[0]) == 1 and not cyc[1:].any()
    u = [0] * n
    u[5] = 1
    v = [0] * n
    v[7] = 3
    assert [int(t) for t in op.negacyclic_conv(u, v, p)] == [3 if i == 12 else 0 for i in range(n)]


def test_eq13_split_of_the_circular_product():
    """eq. 13: Z[x]/(x^2n - 1) = Z[x]/(x^n - 1) x Z[x]/(x^n + 1).  The circular
    product of length 2n, reduced mod x^n - 1 and mod x^n + 1, equals the
    circular and the nega-circular products of the reduced operands."""
    p = 469762049
    rng = np.random.default_rng(32)
    n = 32
    u = rng.integers(0, p, 2 * n, dtype=np.uint32)
    v = rng.integers(0, p, 2 * n, dtype=np.uint32)
    w = op.cyclic_conv(u, v, p)
    assert np.array_equal(op.fold(w, n, p, +1), op.cyclic_conv(op.fold(u, n, p, +1), op.fold(v, n, p, +1), p))
    assert np.array_equal(op.fold(w, n, p, -1), op.negacyclic_conv(op.fold(u, n, p, -1), op.fold(v, n, p, -1), p))


def test_negacyclic_agrees_at_odd_powers_of_psi():
    """The roots of x^N + 1 are the odd powers of a primitive 2N-th root of
    unity psi; there the nega-circular product equals a(x) b(x)."""
    p, g = 2013265921, 31
    n = 64
    rng = np.random.default_rng(33)
    u = rng.integers(0, p, n, dtype=np.uint32)
    v = rng.integers(0, p, n, dtype=np.uint32)
    c = op.negacyclic_conv(u, v, p)
    psi = op.root(p, g, 2 * n)
    for k in (0, 1, 5, 63):
        x = pow(psi, 2 * k + 1, p)
        assert op.eval_at(c, p, x) == op.eval_at(u, p, x) * op.eval_at(v, p, x) % p


def test_multivariate_product_pins():
    """The multivariate product by definition: one variable reduces to the
    univariate schoolbook product; (1+x)^m (1+y)^n has binomial products as
    coefficients; and the product agrees with a(x) b(x) at random points."""
    p = 167772161
    rng = np.random.default_rng(34)
    a = rng.integers(0, p, 37, dtype=np.uint32)
    b = rng.integers(0, p, 21, dtype=np.uint32)
    assert np.array_equal(op.poly_mul_multi(a, b, p), op.poly_mul(a, b, p))
    m, n = 6, 9
    ax = np.array([[math.comb(m, i) * math.comb(n, j) % p for j in range(n + 1)] for i in range(m + 1)])
    c = op.poly_mul_multi(ax, ax, p)
    want = [[math.comb(2 * m, i) * math.comb(2 * n, j) % p for j in range(2 * n + 1)] for i in range(2 * m + 1)]
    assert np.array_equal(c, np.array(want, dtype=np.uint32))
    a = rng.integers(0, p, (3, 4, 5), dtype=np.uint32)
    b = rng.integers(0, p, (2, 6, 3), dtype=np.uint32)
    c = op.poly_mul_multi(a, b, p)
    assert c.shape == (4, 9, 7)
    for _ in range(3):
        xs = [int(t) for t in rng.integers(1, p, 3)]
        assert op.eval_multi(c, p, xs) == op.eval_multi(a, p, xs) * op.eval_multi(b, p, xs) % p


def test_large_ntt_roundtrip_and_theorem():
    p, g = 2013265921, 31
    rng = np.random.default_rng(5)
    n = 1 << 14
    x = rng.integers(0, p, n, dtype=np.uint32)
    X = op.ntt(x, p, g)
    assert np.array_equal(op.ntt(X, p, g, inverse=True), x)
    w = op.root(p, g, n)
    for k in (0, 1, 777, n - 1):
        assert int(X[k]) == op.eval_at(x, p, pow(w, k, p))


def check_tft(tft):
    rec = _records("transform_p17.txt")[0]
    p, g = rec["p"][0], rec["g"][0]
    got = [int(v) for v in tft(rec["tft_in"], len(rec["tft_in"]), rec["tft_L"][0], len(rec["tft_out"]), p, g)]
    assert got == rec["tft_out"]
    for p, g in PRIMES[:2]:
        rng = random.Random(11)
        for L in (1, 2, 8, 32):
            l = L.bit_length() - 1
            w = op.root(p, g, L)
            for z in (1, L // 2 + 1 if L > 1 else 1, L):
                x = [rng.randrange(p) for _ in range(z)]
                for n in sorted({1, max(1, L // 2), max(1, L - 3), L}):
                    out = [int(v) for v in tft(x, z, L, n, p, g)]
                    assert out == [op.eval_at_py(x, p, pow(w, op.bitrev(i, l), p)) for i in range(n)]
            # n = L: the bit-reversed full transform
            x = [rng.randrange(p) for _ in range(L)]
            full = [int(v) for v in op.ntt(x, p, g)]
            assert [int(v) for v in tft(x, L, L, L, p, g)] == [full[op.bitrev(i, l)] for i in range(L)]


def test_tft_pins():
    check_tft(op.tft)


def test_tft_direct_pins():
    check_tft(op.tft_direct)


def test_tft_points_distinct_and_product_recoverable():
    """Any n distinct points fix a polynomial of degree < n: the n TFT points
    are distinct, so pointwise products of two TFTs determine the product
    (the TFT product, eq. 14).  Check by Lagrange interpolation on a tiny case."""
    p, g = 998244353, 3
    L, la, lb = 16, 5, 7
    n = la + lb - 1
    rng = random.Random(2)
    a = [rng.randrange(p) for _ in range(la)]
    b = [rng.randrange(p) for _ in range(lb)]
    ta = op.tft(a, la, L, n, p, g)
    tb = op.tft(b, lb, L, n, p, g)
    w = op.root(p, g, L)
    pts = [pow(w, op.bitrev(i, 4), p) for i in range(n)]
    assert len(set(pts)) == n
    vals = [int(x) * int(y) % p for x, y in zip(ta, tb)]
    # Lagrange interpolation in coefficient form
    coeffs = [0] * n
    for i in range(n):
        num = [1]
        den = 1
        for j in range(n):
            if j == i:
                continue
            num = [((num[k - 1] if k > 0 else 0) - pts[j] * (num[k] if k < len(num) else 0)) % p for k in range(len(num) + 1)]
            den = den * (pts[i] - pts[j]) % p
        f = vals[i] * pow(den, p - 2, p) % p
        for k in range(n):
            coeffs[k] = (coeffs[k] + f * num[k]) % p
    assert coeffs == kronecker_product(a, b, p)


# --- three-primes pins ----------------------------------------------------------

def test_crt_fixture_and_forms():
    rec = _records("crt_small.txt")[0]
    assert op.crt3(rec["residues"], rec["primes"]) == rec["x"][0]
    assert op.crt3_garner(rec["residues"], rec["primes"]) == rec["x"][0]
    P = inputs.INT_PRIMES
    M = P[0] * P[1] * P[2]
    assert M == 78674626319836206717730817
    rng = random.Random(4)
    for _ in range(200):
        x = rng.randrange(M)
        r = [x % q for q in P]
        assert op.crt3(r, P) == x
        assert op.crt3_garner(r, P) == x
    for x in (0, 1, M - 1, 2 ** 53):
        assert op.crt3([x % q for q in P], P) == x


def check_int_mul(mul):
    rng = np.random.default_rng(8)
    for na, nb in ((1, 1), (3, 2), (17, 40), (256, 255)):
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        want = op.carry_limbs(op.int_convolve(a, b), na + nb)
        assert np.array_equal(mul(a, b), want)
    # (2^(16n) - 1)^2 = limbs [1, 0 x (n-1), 0xFFFE, 0xFFFF x (n-1)]
    n = 64
    ff = np.full(n, 0xFFFF, dtype=np.uint16)
    want = np.array([1] + [0] * (n - 1) + [0xFFFE] + [0xFFFF] * (n - 1), dtype=np.uint16)
    assert np.array_equal(mul(ff, ff), want)
    # reduction mod a random 61-bit modulus commutes with the product
    a = rng.integers(0, 1 << 16, 5000, dtype=np.uint16)
    b = rng.integers(0, 1 << 16, 3000, dtype=np.uint16)
    c = mul(a, b)
    q = (1 << 61) - 1
    assert op.limbs_to_int(c) % q == (op.limbs_to_int(a) % q) * (op.limbs_to_int(b) % q) % q


def test_int_mul_pins():
    check_int_mul(op.int_mul)


def test_crt_bound_for_int_products():
    """The exact coefficient sums of 2^21-limb products stay below p1 p2 p3."""
    P = inputs.INT_PRIMES
    assert (1 << 21) * (0xFFFF ** 2) < P[0] * P[1] * P[2]
    # and the transform length 2^22 divides p - 1 for each of the three primes
    for q in P:
        assert (q - 1) % (1 << 22) == 0


def test_crt_bound_for_32_bit_digits():
    """Pairs of limbs as 32-bit digits: for every supported size (na + nb - 1
    <= 2^23 limbs, so at most 2^21 digits in the shorter operand) the exact
    digit-product sums stay below p1 p2 p3, and the transform length (at
    most 2^22 points) divides p - 1 for each prime; the digits' convolution,
    summed at 2^32 per position, is the integer product (checked exactly on
    small operands, odd limb counts included, by CPython integers)."""
    P = inputs.INT_PRIMES
    assert (1 << 21) * (0xFFFFFFFF ** 2) < P[0] * P[1] * P[2]
    for q in P:
        assert (q - 1) % (1 << 22) == 0
    rng = np.random.default_rng(81)
    for na, nb in ((1, 1), (3, 2), (17, 40), (255, 256), (1001, 998)):
        a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
        b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
        da = [int(a[2 * j]) + (int(a[2 * j + 1]) << 16 if 2 * j + 1 < na else 0) for j in range((na + 1) // 2)]
        db = [int(b[2 * j]) + (int(b[2 * j + 1]) << 16 if 2 * j + 1 < nb else 0) for j in range((nb + 1) // 2)]
        x = [0] * (len(da) + len(db) - 1)
        for i, u in enumerate(da):
            for j, v in enumerate(db):
                x[i + j] += u * v
        assert max(x) < min(len(da), len(db)) * (1 << 64)
        value = sum(xk << (32 * k) for k, xk in enumerate(x))
        assert value == op.limbs_to_int(a) * op.limbs_to_int(b)
        assert np.array_equal(op.int_mul(a, b), op.carry_limbs(op.int_convolve(a, b), na + nb))


# --- cost-model network pins ------------------------------------------------------

def _mlp_params(F=7, H=16, seed=0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, 0.5, (H, F)), "b1": rng.normal(0, 0.1, H),
        "W2": rng.normal(0, 0.3, (H, H)), "b2": rng.normal(0, 0.1, H),
        "W3": rng.normal(0, 0.3, (1, H)), "b3": rng.normal(0, 0.1, 1),
    }


def check_mlp_grad(backward):
    params = _mlp_params()
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (9, 7))
    t = rng.normal(0, 1, 9)
    g = backward(params, X, t)
    eps = 1e-6
    for k in omlp.NAMES:
        flat = params[k].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + eps
            lp = omlp.loss(params, X, t)
            flat[idx] = old - eps
            lm = omlp.loss(params, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_mlp_gradient_finite_differences():
    check_mlp_grad(omlp.backward)


def test_mlp_closed_forms():
    # zero weights: the output is b3 everywhere; loss gradient wrt b3 = 2 mean(b3 - t)
    F, H = 5, 8
    params = {"W1": np.zeros((H, F)), "b1": np.zeros(H), "W2": np.zeros((H, H)), "b2": np.zeros(H),
              "W3": np.zeros((1, H)), "b3": np.array([0.5])}
    X = np.ones((4, F))
    t = np.array([0.0, 1.0, 2.0, 3.0])
    y, _ = omlp.forward(params, X)
    assert np.allclose(y, 0.5)
    g = omlp.backward(params, X, t)
    assert np.isclose(g["b3"][0], 2 * np.mean(0.5 - t))
    assert np.allclose(g["W1"], 0) and np.allclose(g["W2"], 0)
    # first Adam step moves each parameter by lr * g / (|g| + eps) (bias-corrected)
    p2 = {k: v.copy() for k, v in params.items()}
    omlp.adam_step(p2, g, {}, lr=0.01)
    assert np.isclose(p2["b3"][0], 0.5 - 0.01 * np.sign(g["b3"][0]) * abs(g["b3"][0]) / (abs(g["b3"][0]) + 1e-8))


def _adam_case():
    """Parameters and two gradients per element for the Adam pins.  W1 row 0:
    the same gradient twice; row 1: g then -g; row 2: g then 0.  The other
    tensors get the same gradient at both steps."""
    F, H = 3, 4
    g1 = np.array([[0.5, -2.0, 3e-3], [1.5, -0.25, 7.0], [2.0, -0.75, 0.125], [1.0, 1.0, -1.0]])
    g2 = g1.copy()
    g2[1] = -g1[1]
    g2[2] = 0.0
    params = {"W1": np.full((H, F), 0.25), "b1": np.zeros(H), "W2": np.eye(H), "b2": np.ones(H),
              "W3": np.ones((1, H)), "b3": np.array([0.5])}
    grads1 = {"W1": g1, "b1": np.full(H, -0.5), "W2": np.full((H, H), 2.0), "b2": np.full(H, 4.0),
              "W3": np.full((1, H), -1.0), "b3": np.array([0.01])}
    grads2 = dict(grads1, W1=g2)
    return params, grads1, grads2


def check_adam(step_fn, lr=0.01, eps=1e-8):
    """Adam with bias correction (beta1 0.9, beta2 0.999), pinned by values
    derived by hand from the moments' closed forms:
      - a gradient g held for t steps: m_t = (1 - beta1^t) g and
        v_t = (1 - beta2^t) g^2, so every step moves by lr g / (|g| + eps);
      - g then -g: m_2 = -(1 - beta1)^2 g, so m_2 / (1 - beta1^2) = -g/19,
        and v_2 / (1 - beta2^2) = g^2: the second step moves by
        +lr g / (19 (|g| + eps));
      - g then 0: the corrected moments are 9/19 g and 999/1999 g^2, so the
        second step moves by -lr (9/19) g / (sqrt(999/1999) |g| + eps)."""
    params, grads1, grads2 = _adam_case()
    p = {k: v.copy() for k, v in params.items()}
    state = {}
    step_fn(p, grads1, state, lr=lr)
    for k in omlp.NAMES:
        g = grads1[k]
        assert np.allclose(p[k], params[k] - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12), ("step 1", k)
    after1 = {k: np.array(v, dtype=np.float64) for k, v in p.items()}
    step_fn(p, grads2, state, lr=lr)
    g = grads1["W1"]
    want = after1["W1"].copy()
    want[0] -= lr * g[0] / (np.abs(g[0]) + eps)
    want[1] += lr * g[1] / (19.0 * (np.abs(g[1]) + eps))
    want[2] -= lr * (9.0 / 19.0) * g[2] / (math.sqrt(999.0 / 1999.0) * np.abs(g[2]) + eps)
    want[3] -= lr * g[3] / (np.abs(g[3]) + eps)
    assert np.allclose(p["W1"], want, rtol=0, atol=1e-12), "step 2, W1"
    for k in omlp.NAMES[1:]:
        gk = grads1[k]
        assert np.allclose(p[k], after1[k] - lr * gk / (np.abs(gk) + eps), rtol=0, atol=1e-12), ("step 2", k)
    # three more steps of a constant gradient: each moves by lr g / (|g| + eps)
    p = {k: v.copy() for k, v in params.items()}
    state = {}
    for _ in range(5):
        step_fn(p, grads1, state, lr=lr)
    for k in omlp.NAMES:
        g = grads1[k]
        assert np.allclose(p[k], params[k] - 5 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-11), ("step 5", k)


def test_adam_steps_match_closed_forms():
    check_adam(omlp.adam_step)


def test_mlp_training_reduces_loss():
    params = _mlp_params(F=3, H=16, seed=3)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (64, 3))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    l0 = omlp.loss(params, X, t)
    trained = omlp.train(params, X, t, steps=300, lr=3e-3)
    assert omlp.loss(trained, X, t) < 0.2 * l0


# --- planted mistakes: each must be caught by a pin above -------------------------

def _mutant_dropped_term(a, b, p):
    c = op.poly_mul_py(a, b, p)
    if len(a) > 2 and len(b) > 1:   # drops a_1 b_1 from c_2
        c[2] = (c[2] - int(a[1]) * int(b[1])) % p
    return c


def _mutant_index_shift(a, b, p):
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    c = [0] * (len(a) + len(b) - 1)
    for i in range(len(a)):
        for j in range(len(b)):
            c[min(i + j + (1 if i == len(a) - 1 and j > 0 else 0), len(c) - 1)] += a[i] * b[j]
    return [x % p for x in c]


def _mutant_reversed_operand(a, b, p):
    return op.poly_mul_py(a, list(reversed(list(b))), p)


def _mutant_no_reduction_of_last(a, b, p):
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    c = [0] * (len(a) + len(b) - 1)
    for i in range(len(a)):
        for j in range(len(b)):
            c[i + j] += a[i] * b[j]
    return [x % p for x in c[:-1]] + [c[-1] % (2 ** 32)]


@pytest.mark.parametrize("mutant", [_mutant_dropped_term, _mutant_index_shift, _mutant_reversed_operand,
                                    _mutant_no_reduction_of_last])
def test_product_pins_catch_mistakes(mutant):
    with pytest.raises(AssertionError):
        check_product(mutant)


def _ntt_wrong_sign(x, p, g, inverse):
    return op.ntt(x, p, g, not inverse) if len(x) > 2 else op.ntt(x, p, g, inverse)


def _ntt_no_scale(x, p, g, inverse):
    y = op.ntt(x, p, g, inverse)
    if inverse:
        n = len(x)
        y = [int(v) * n % p for v in y]
    return y


def _ntt_bitrev_out(x, p, g, inverse):
    y = op.ntt(x, p, g, inverse)
    n = len(y)
    l = n.bit_length() - 1
    return [y[op.bitrev(i, l)] for i in range(n)]


@pytest.mark.parametrize("mutant", [_ntt_wrong_sign, _ntt_no_scale, _ntt_bitrev_out])
def test_ntt_pins_catch_mistakes(mutant):
    with pytest.raises(AssertionError):
        check_ntt(mutant)


def _tft_natural_order(x, z, L, n, p, g):
    buf = list(x[:z]) + [0] * (L - z)
    return op.ntt(buf, p, g)[:n]


def _tft_ignores_z(x, z, L, n, p, g):
    return op.tft(x[: max(1, z - 1)], max(1, z - 1), L, n, p, g)


@pytest.mark.parametrize("mutant", [_tft_natural_order, _tft_ignores_z])
def test_tft_pins_catch_mistakes(mutant):
    with pytest.raises(AssertionError):
        check_tft(mutant)


def _int_mul_dropped_carry(a, b):
    c = op.int_convolve(a, b)
    out = [int(v) & 0xFFFF for v in c] + [0]
    return np.array(out, dtype=np.uint16)


def _int_mul_short_output(a, b):
    x = op.limbs_to_int(a) * op.limbs_to_int(b)
    n = len(a) + len(b)
    return op.int_to_limbs(x % (1 << (16 * (n - 1))), n - 1)


@pytest.mark.parametrize("mutant", [_int_mul_dropped_carry, _int_mul_short_output])
def test_int_pins_catch_mistakes(mutant):
    with pytest.raises((AssertionError, ValueError)):
        check_int_mul(mutant)


def _backward_missing_tanh_derivative(params, X, t):
    g = omlp.backward(params, X, t)
    W2 = params["W2"]
    W3 = params["W3"]
    y, (Xc, h1, h2) = omlp.forward(params, X)
    dy = 2.0 * (y - t) / X.shape[0]
    dz2 = dy[:, None] * W3
    g["W2"] = dz2.T @ h1
    return g


def _backward_transposed(params, X, t):
    g = omlp.backward(params, X, t)
    g["W2"] = g["W2"].T
    return g


@pytest.mark.parametrize("mutant", [_backward_missing_tanh_derivative, _backward_transposed])
def test_mlp_pins_catch_mistakes(mutant):
    with pytest.raises(AssertionError):
        check_mlp_grad(mutant)


def _adam_variant(bias_t=None, persist=True, betas=(0.9, 0.999)):
    """A copy of the oracle's Adam step with one planted change."""
    def step(params, grads, state, lr=1e-3, eps=1e-8):
        beta1, beta2 = betas
        state["t"] = state.get("t", 0) + 1
        tt = state["t"] if bias_t is None else bias_t
        if not persist:
            state["m"], state["v"] = {}, {}
        for k in omlp.NAMES:
            g = np.asarray(grads[k], dtype=np.float64)
            m = state.setdefault("m", {}).setdefault(k, np.zeros_like(g))
            v = state.setdefault("v", {}).setdefault(k, np.zeros_like(g))
            m[...] = beta1 * m + (1.0 - beta1) * g
            v[...] = beta2 * v + (1.0 - beta2) * g * g
            mhat = m / (1.0 - beta1 ** tt)
            vhat = v / (1.0 - beta2 ** tt)
            params[k] = np.asarray(params[k], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        return params
    return step


@pytest.mark.parametrize("mutant", [_adam_variant(bias_t=1), _adam_variant(persist=False),
                                    _adam_variant(betas=(0.999, 0.9))],
                         ids=["bias_correction_stuck_at_t1", "moments_not_persisted", "betas_swapped"])
def test_adam_pins_catch_mistakes(mutant):
    # the unmodified copy passes: the pins see only the planted change
    check_adam(_adam_variant())
    with pytest.raises(AssertionError):
        check_adam(mutant)
