"""Plain, slow, obviously correct modular polynomial arithmetic on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions fixed here, where the paper leaves a choice open:
  * a polynomial is its coefficient array, index i = coefficient of x^i
    (Def. 1); the product of lengths la and lb has la + lb - 1 coefficients
    (Def. 2 indexes degrees n, m and returns m + n + 1 of them; the "< M+N"
    bound printed with eq. 3 is read as "<= M+N-2");
  * the length-N transform uses w_N = g^((p-1)/N) for the primitive root g of
    each prime (the paper fixes no root);
  * the TFT returns the first n values in bit-reversed order: out_i is the
    input polynomial evaluated at w_L^{rev_l(i)}, l = log2 L (the paper says
    "the first n Fourier coefficients" without naming the order);
  * the ITFT of the TFT product returns L times the coefficients (it yields
    (L u_0, ..., L u_{n-1})); the second TFT of the product applies to h,
    not g (a misprint in the statement of the TFT product).
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

from ._clib import lib

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _as_u32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


# --- roots of unity -----------------------------------------------------------

def root(p: int, g: int, n: int, inverse: bool = False) -> int:
    """w_n = g^((p-1)/n) mod p, a primitive n-th root of unity when n | p-1."""
    if (p - 1) % n:
        raise ValueError("n does not divide p-1")
    w = pow(g, (p - 1) // n, p)
    return pow(w, p - 2, p) if inverse else w


def bitrev(i: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


# --- products -----------------------------------------------------------------

def poly_mul(a, b, p: int) -> np.ndarray:
    """c_k = sum_{i+j=k} a_i b_j mod p for 0 <= k <= la+lb-2 (Def. 2, eq. 2).

    Schoolbook sum over the output index in C with 128-bit accumulation."""
    a = _as_u32(a)
    b = _as_u32(b)
    if a.size == 0 or b.size == 0:
        raise ValueError("empty operand")
    c = np.zeros(a.size + b.size - 1, dtype=np.uint32)
    lib().orc_polymul(_ptr(a), a.size, _ptr(b), b.size, p, _ptr(c))
    return c


def poly_mul_py(a, b, p: int) -> list:
    """The same sum with Python integers (tiny inputs only)."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    c = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            c[i + j] += ai * bj
    return [x % p for x in c]


def poly_mul_sample(a, b, p: int, ks) -> np.ndarray:
    """Coefficients c_k of a*b mod p for the given output indices only (Def. 2)."""
    a = _as_u32(a)
    b = _as_u32(b)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    lc = a.size + b.size - 1
    if ks.size and (ks.min() < 0 or ks.max() >= lc):
        raise ValueError("index out of range")
    out = np.zeros(ks.size, dtype=np.uint32)
    lib().orc_polymul_sample(_ptr(a), a.size, _ptr(b), b.size, p, ks.ctypes.data_as(_i64p), ks.size, _ptr(out))
    return out


def poly_mul_ntt(a, b, p: int, g: int) -> np.ndarray:
    """a*b mod p by zero padding to a power of two and the textbook radix-2
    transform (eq. 12).  Faster than the schoolbook sum; pinned against it."""
    a = _as_u32(a)
    b = _as_u32(b)
    c = np.zeros(a.size + b.size - 1, dtype=np.uint32)
    rc = lib().orc_polymul_ntt(_ptr(a), a.size, _ptr(b), b.size, p, g, _ptr(c))
    if rc:
        raise ValueError("transform length not supported by p (rc=%d)" % rc)
    return c


def cyclic_conv(u, v, p: int) -> np.ndarray:
    """(u (*) v)_i = sum_k u_k v_{(i-k) mod N} mod p (Def. 4, eq. 5)."""
    u = _as_u32(u)
    v = _as_u32(v)
    if u.size != v.size:
        raise ValueError("lengths differ")
    out = np.zeros(u.size, dtype=np.uint32)
    lib().orc_cyclic(_ptr(u), _ptr(v), u.size, p, _ptr(out))
    return out


def negacyclic_conv(u, v, p: int) -> np.ndarray:
    """u v mod (x^N + 1) mod p by its defining sums (the nega-circular factor of eq. 13)."""
    u = _as_u32(u)
    v = _as_u32(v)
    if u.size != v.size:
        raise ValueError("lengths differ")
    out = np.zeros(u.size, dtype=np.uint32)
    lib().orc_negacyclic(_ptr(u), _ptr(v), u.size, p, _ptr(out))
    return out


def poly_mul_multi(a, b, p: int) -> np.ndarray:
    """Dense multivariate product by its definition: c[e + f] += a[e] b[f] mod p
    (arrays indexed by exponent vectors, one axis per variable)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    c = np.zeros(tuple(x + y - 1 for x, y in zip(a.shape, b.shape)), dtype=np.int64)
    for e in np.ndindex(*a.shape):
        if a[e]:
            box = tuple(slice(ei, ei + bi) for ei, bi in zip(e, b.shape))
            c[box] = (c[box] + a[e] * b) % p
    return c.astype(np.uint32)


def eval_multi(a, p: int, xs) -> int:
    """a(x_1, .., x_k) mod p for an array a indexed by exponent vectors."""
    a = np.asarray(a, dtype=np.int64)
    total = 0
    for e in np.ndindex(*a.shape):
        t = int(a[e])
        for ei, x in zip(e, xs):
            t = t * pow(x, ei, p) % p
        total = (total + t) % p
    return total


def fold(c, n: int, p: int, sign: int) -> np.ndarray:
    """Reduce the coefficients c of a polynomial mod x^n - sign (sign = +1 or -1):
    out_i = sum_m sign^m c_{i + m n} mod p."""
    c = np.asarray(c, dtype=np.int64)
    out = np.zeros(n, dtype=np.int64)
    for m in range(0, (c.size + n - 1) // n):
        blk = c[m * n:(m + 1) * n]
        s = 1 if (sign == 1 or m % 2 == 0) else -1
        out[:blk.size] = (out[:blk.size] + s * blk) % p
    return (out % p).astype(np.uint32)


def eval_at(a, p: int, x: int) -> int:
    """a(x) mod p by Horner's rule."""
    a = _as_u32(a)
    return int(lib().orc_eval(_ptr(a), a.size, p, x))


def eval_at_py(a, p: int, x: int) -> int:
    r = 0
    for c in reversed([int(v) for v in a]):
        r = (r * x + c) % p
    return r


# --- transforms ---------------------------------------------------------------

def dft_direct(x, p: int, g: int, inverse: bool = False) -> list:
    """X_k = sum_j x_j w^{jk} mod p, the evaluation of x at w^0..w^{N-1}
    (section 3); with inverse, w^-1 and a factor N^-1.  O(N^2), Python ints."""
    x = [int(v) for v in x]
    n = len(x)
    w = root(p, g, n, inverse)
    out = []
    for k in range(n):
        wk = pow(w, k, p)
        acc = 0
        t = 1
        for xj in x:
            acc += xj * t
            t = t * wk % p
        out.append(acc % p)
    if inverse:
        ninv = pow(n, p - 2, p)
        out = [v * ninv % p for v in out]
    return out


def dft_eval(x, p: int, g: int, inverse: bool = False, ks=None) -> np.ndarray:
    """X_k = x(w^k) mod p for a length N = len(x) dividing p - 1, any N (section
    3: the transform evaluates x at w^0 .. w^{N-1}, w = g^((p-1)/N)); with
    inverse, x(w^-k) N^-1.  Only the indices ks (all by default), each by
    Horner's rule: O(N) per value."""
    x = _as_u32(x)
    n = x.size
    w = root(p, g, n, inverse)
    ks = range(n) if ks is None else ks
    out = np.array([eval_at(x, p, pow(w, int(k), p)) for k in ks], dtype=np.uint64)
    if inverse:
        out = out * pow(n, p - 2, p) % p
    return out.astype(np.uint32)


def ntt(x, p: int, g: int, inverse: bool = False) -> np.ndarray:
    """Length-N transform in natural order by the iterative radix-2 algorithm
    (C); inverse includes N^-1.  Pinned against dft_direct."""
    y = _as_u32(x).copy()
    rc = lib().orc_ntt(_ptr(y), y.size, p, g, 1 if inverse else 0)
    if rc:
        raise ValueError("length not supported (rc=%d)" % rc)
    return y


def tft_direct(x, z: int, L: int, n: int, p: int, g: int) -> list:
    """out_i = sum_{j<z} x_j w_L^{j rev_l(i)} for i < n: the first n values of
    the length-L transform of (x_0..x_{z-1}) in bit-reversed order (TFT(L, z, n))."""
    l = L.bit_length() - 1
    if 1 << l != L or z > L or n > L:
        raise ValueError("bad TFT sizes")
    w = root(p, g, L)
    xs = [int(v) for v in x[:z]]
    out = []
    for i in range(n):
        pt = pow(w, bitrev(i, l), p)
        out.append(eval_at_py(xs, p, pt))
    return out


def tft(x, z: int, L: int, n: int, p: int, g: int) -> np.ndarray:
    """TFT(L, z, n) by a full length-L transform of the zero-padded input,
    reordered bit-reversed and cut to n values.  Pinned against tft_direct."""
    l = L.bit_length() - 1
    if 1 << l != L or z > L or n > L:
        raise ValueError("bad TFT sizes")
    buf = np.zeros(L, dtype=np.uint32)
    buf[:z] = _as_u32(x)[:z]
    full = ntt(buf, p, g)
    return full[bitrev_perm(L)[:n]]


# --- three-primes integer product (section 1) ---------------------------------

def crt3(r, primes) -> int:
    """The unique x in [0, p1 p2 p3) with x = r_i mod p_i, by the sum form
    x = sum_i r_i M_i (M_i^-1 mod p_i) mod M."""
    M = 1
    for q in primes:
        M *= q
    x = 0
    for ri, q in zip(r, primes):
        Mi = M // q
        x += int(ri) * Mi * pow(Mi, -1, q)
    return x % M


def crt3_garner(r, primes) -> int:
    """The same value by Garner's mixed-radix recurrence."""
    p1, p2, p3 = primes
    v1 = int(r[0]) % p1
    v2 = (int(r[1]) - v1) * pow(p1, -1, p2) % p2
    v3 = (int(r[2]) - v1 - p1 * v2) * pow(p1 * p2, -1, p3) % p3
    return v1 + p1 * v2 + p1 * p2 * v3


def limbs_to_int(limbs) -> int:
    a = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint16))
    return int.from_bytes(a.astype("<u2").tobytes(), "little")


def int_to_limbs(x: int, n: int) -> np.ndarray:
    if x < 0 or x.bit_length() > 16 * n:
        raise ValueError("value does not fit")
    return np.frombuffer(x.to_bytes(2 * n, "little"), dtype="<u2").astype(np.uint16)


def int_mul(a_limbs, b_limbs) -> np.ndarray:
    """The product of two little-endian 16-bit-limb integers, as na+nb limbs
    (fixed length; the top limb may be 0), by CPython's integer multiply."""
    na = len(a_limbs)
    nb = len(b_limbs)
    return int_to_limbs(limbs_to_int(a_limbs) * limbs_to_int(b_limbs), na + nb)


def carry_limbs(coeffs, n: int) -> np.ndarray:
    """Limbs of sum_k coeffs_k 2^{16k}: add each coefficient at its position
    and propagate carries one limb at a time (Python ints)."""
    out = [0] * n
    carry = 0
    for k in range(n):
        v = carry + (int(coeffs[k]) if k < len(coeffs) else 0)
        out[k] = v & 0xFFFF
        carry = v >> 16
    if carry:
        raise ValueError("carry out of the top limb")
    return np.array(out, dtype=np.uint16)


def int_convolve(a_limbs, b_limbs) -> list:
    """Exact (non-modular) coefficient sums sum_{i+j=k} a_i b_j, Python ints."""
    a = [int(v) for v in a_limbs]
    b = [int(v) for v in b_limbs]
    c = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai:
            for j, bj in enumerate(b):
                c[i + j] += ai * bj
    return c


def bitrev_perm(L: int) -> np.ndarray:
    """[rev_l(i) for i < L], built bit by bit with numpy."""
    l = L.bit_length() - 1
    i = np.arange(L, dtype=np.int64)
    r = np.zeros(L, dtype=np.int64)
    for _ in range(l):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def binom_mod(n: int, k: int, p: int) -> int:
    return math.comb(n, k) % p
