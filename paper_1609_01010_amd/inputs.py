"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module only draws numbers: it holds none of the method's arithmetic, so
the HIP path and the CPU oracle can both be fed from it without sharing any
computation.  Every draw uses numpy's PCG64 seeded with ``[160901010, tag]``
and happens in the order written here, so a workload is fully determined by
its tag.

The paper measures on no public dataset (its Fig. 3 lengths are not printed);
the workloads below are the synthetic stand-ins: coefficients uniform in
[0, p) for the modular products, uniform 16-bit limbs for the integer product.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 160901010

# The four NTT-friendly primes and a primitive root of each: p - 1 = c * 2^k.
PRIMES = {
    998244353: 3,      # 119 * 2^23 + 1
    2013265921: 31,    # 15 * 2^27 + 1
    469762049: 3,      # 7 * 2^26 + 1
    167772161: 3,      # 5 * 2^25 + 1
}
PRIME_LIST = (998244353, 2013265921, 469762049, 167772161)
# primes of the three-primes integer product, in CRT order
INT_PRIMES = (469762049, 998244353, 167772161)


def rng_for(tag) -> np.random.Generator:
    """Generator for one workload; ``tag`` is an int or a tuple of ints."""
    if isinstance(tag, (tuple, list)):
        key = [SEED_BASE, *[int(t) for t in tag]]
    else:
        key = [SEED_BASE, int(tag)]
    return np.random.Generator(np.random.PCG64(key))


def uniform_mod(rng: np.random.Generator, n: int, p: int) -> np.ndarray:
    """n coefficients uniform in [0, p) as uint32."""
    return rng.integers(0, p, size=n, dtype=np.uint32)


def poly_pair(tag, la: int, lb: int, p: int):
    """Two random polynomials (a then b) with uniform coefficients mod p."""
    rng = rng_for(tag)
    a = uniform_mod(rng, la, p)
    b = uniform_mod(rng, lb, p)
    return a, b


# --- the five workloads -------------------------------------------------------

def single_product_1024():
    """Plain single product: 1024 x 1024 coefficients mod 998244353 (cyclic size 2048)."""
    p = 998244353
    a, b = poly_pair(1, 1024, 1024, p)
    return a, b, p


def large_pow2_product():
    """Two length-2^21 polynomials mod 2013265921 (transform size 2^22)."""
    p = 2013265921
    a, b = poly_pair((2, 1), 1 << 21, 1 << 21, p)
    return a, b, p


def large_tft_product():
    """Lengths 600001 and 400000 mod 2013265921: 1000000 output coefficients."""
    p = 2013265921
    a, b = poly_pair((2, 2), 600001, 400000, p)
    return a, b, p


def int_operands(n_limbs: int = 1 << 21, tag=3):
    """Two random integers of n_limbs 16-bit limbs each (little-endian, uniform)."""
    rng = rng_for(tag)
    a = rng.integers(0, 1 << 16, size=n_limbs, dtype=np.uint16)
    b = rng.integers(0, 1 << 16, size=n_limbs, dtype=np.uint16)
    return a, b


def log_uniform_len(rng: np.random.Generator, lo: int, hi: int, size: int) -> np.ndarray:
    """floor(exp(U[ln lo, ln(hi + 1)))), so every length in [lo, hi] can occur."""
    u = rng.uniform(math.log(lo), math.log(hi + 1), size=size)
    out = np.floor(np.exp(u)).astype(np.int64)
    return np.clip(out, lo, hi)


@dataclass
class BatchItem:
    a: np.ndarray
    b: np.ndarray
    p: int


def batch_uneven(count: int = 4096, lo: int = 64, hi: int = 65536, tag=4):
    """Independent products: lengths log-uniform in [lo, hi], prime uniform over the four.

    Draw order: all len_a, all len_b, all prime indices, then the coefficients
    of a and b product by product.
    """
    rng = rng_for(tag)
    la = log_uniform_len(rng, lo, hi, count)
    lb = log_uniform_len(rng, lo, hi, count)
    pidx = rng.integers(0, len(PRIME_LIST), size=count)
    items = []
    for i in range(count):
        p = PRIME_LIST[int(pidx[i])]
        a = uniform_mod(rng, int(la[i]), p)
        b = uniform_mod(rng, int(lb[i]), p)
        items.append(BatchItem(a, b, p))
    return items


def tuning_lengths(tag=5, n_random: int = 300, lo_log: int = 10, hi_log: int = 20, n_large: int = 60,
                   large_hi_log: int = 23):
    """Output lengths the tuner measures: every power of two 2^lo..2^hi, plus
    n_random non-power-of-two lengths log-uniform in [2^lo, 2^hi], plus
    n_large non-power-of-two lengths log-uniform in [2^hi, 2^large_hi] (no
    powers of two there: 2^21.. stay held out)."""
    rng = rng_for(tag)
    pow2 = [1 << k for k in range(lo_log, hi_log + 1)]
    rnd = log_uniform_len(rng, 1 << lo_log, 1 << hi_log, n_random * 2)
    rnd = [int(x) for x in rnd if int(x) & (int(x) - 1)]
    seen = set(pow2)
    out = list(pow2)
    for x in rnd:
        if x not in seen:
            seen.add(x)
            out.append(x)
        if len(out) >= len(pow2) + n_random:
            break
    want = len(out) + n_large
    big = rng_for((tag, 1))
    while len(out) < want:
        for x in log_uniform_len(big, 1 << hi_log, 1 << large_hi_log, 64):
            x = int(x)
            if x & (x - 1) and x not in seen:
                seen.add(x)
                out.append(x)
                if len(out) >= want:
                    break
    return out


def heldout_lengths(tag=6, n_random: int = 200, exclude=(), lo_log: int = 10, hi_log: int = 24):
    """Held-out output lengths: the powers of two 2^21..2^24 plus n_random
    non-power-of-two lengths log-uniform in [2^lo, 2^hi] not in ``exclude``."""
    rng = rng_for(tag)
    ex = set(int(x) for x in exclude)
    out = [1 << k for k in range(21, 25)]
    seen = set(out) | ex
    while len(out) < 4 + n_random:
        for x in log_uniform_len(rng, 1 << lo_log, 1 << hi_log, 64):
            x = int(x)
            if x & (x - 1) and x not in seen:
                seen.add(x)
                out.append(x)
                if len(out) >= 4 + n_random:
                    break
    return out


def split_output_length(lc: int):
    """Operand lengths (la, lb) with la + lb - 1 = lc and la >= lb."""
    la = (lc + 2) // 2
    lb = lc + 1 - la
    return la, lb


# --- cost-model initial weights -------------------------------------------------

MLP_F, MLP_H = 17, 64


def mlp_init(tag=7):
    """Glorot-uniform initial weights of the cost model, flattened in the
    library's layout W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3 (float32)."""
    rng = rng_for(tag)
    F, H = MLP_F, MLP_H
    a1 = math.sqrt(6.0 / (F + H))
    a2 = math.sqrt(6.0 / (2 * H))
    a3 = math.sqrt(6.0 / (H + 1))
    parts = [rng.uniform(-a1, a1, H * F), np.zeros(H), rng.uniform(-a2, a2, H * H), np.zeros(H),
             rng.uniform(-a3, a3, H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def mlp_unflatten(w):
    """The flat weight vector as the float64 dict the oracle network uses."""
    F, H = MLP_F, MLP_H
    w = np.asarray(w, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out
