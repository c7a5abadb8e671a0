"""The allocation-free product (pm_poly_mul_noalloc) through the C ABI against
pm_poly_mul, bit-exact, on consecutive calls that share the static scratch
array: a larger product, then a smaller one, then sizes of every plan kind,
and the host-side refusal of a product that needs more than the array.

Runs alone in a fresh process and after the other tests (pm_init is called
first either way)."""

import ctypes
import sys

import numpy as np
import pytest

from oracle import poly as op
from paper_1609_01010_amd import inputs

pytestmark = pytest.mark.gpu

PM_OK, PM_EINVAL, PM_ETOOLARGE = 0, 1, 3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _noalloc(pm, ta, tb, p, tc):
    import torch

    L = pm.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.pm_poly_mul_noalloc(ctypes.c_void_p(ta.data_ptr()), ta.numel(), ctypes.c_void_p(tb.data_ptr()),
                                 tb.numel(), p, ctypes.c_void_p(tc.data_ptr()), s)


def test_noalloc_matches_pm_poly_mul_on_consecutive_calls(gpu_lib):
    import torch

    pm = gpu_lib
    assert pm.lib().pm_init() == PM_OK
    pm.set_policy(pm.POLICY_DEFAULT)
    pm.plan_cache_clear()
    # first a product with a relaxed transform of about 2^20 points (four-step,
    # nearly the whole workspace), then a smaller four-step product, then the
    # one-work-group and defining-sum sizes, then the first size again
    cases = [(600001, 400000, 2013265921), (70001, 30000, 998244353), (3000, 1777, 469762049),
             (20, 9, 167772161), (1 << 20, (1 << 20) + 1, 998244353), (600001, 400000, 2013265921)]
    for i, (la, lb, p) in enumerate(cases):
        say("case: noalloc", i, la, lb, p)
        a, b = inputs.poly_pair((190, i), la, lb, p)
        ta, tb = _dev(a), _dev(b)
        want = pm.poly_mul(ta, tb, p)
        got = torch.full((la + lb - 1,), 0xFFFFFFFF, dtype=torch.uint32, device="cuda")
        assert _noalloc(pm, ta, tb, p, got) == PM_OK
        assert pm.stream_check() == 0
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(g, w), f"case {i}: differs from pm_poly_mul at {np.flatnonzero(g != w)[:8]}"
        rng = np.random.default_rng(i)
        ks = np.unique(np.concatenate([[0, la + lb - 2], rng.integers(0, la + lb - 1, 16)]))
        assert np.array_equal(g[ks], op.poly_mul_sample(a, b, p, ks))


def test_noalloc_refuses_products_beyond_its_scratch(gpu_lib):
    import torch

    pm = gpu_lib
    assert pm.lib().pm_init() == PM_OK
    pm.set_policy(pm.POLICY_DEFAULT)
    pm.plan_cache_clear()
    say("case: noalloc too large")
    la = lb = (1 << 20) + 1  # 2^21 + 1 outputs: L = 2^22, beyond the scratch
    ta = torch.zeros(la, dtype=torch.uint32, device="cuda")
    tb = torch.zeros(lb, dtype=torch.uint32, device="cuda")
    tc = torch.full((la + lb - 1,), 7, dtype=torch.uint32, device="cuda")
    assert _noalloc(pm, ta, tb, 998244353, tc) == PM_ETOOLARGE
    torch.cuda.synchronize()
    assert np.all(tc.cpu().numpy() == 7)  # nothing launched
