"""The C ABI on the CPU: the library loads, exports every declared symbol,
and rejects bad arguments on the host before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polymul.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1609_01010_amd as pm

    return pm.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pm_poly_mul", "pm_poly_mul_batch", "pm_int_mul", "pm_ntt", "pm_tft", "pm_itft",
                 "pm_stream_check", "pm_status_str", "pm_set_policy", "pm_plan_for"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    import paper_1609_01010_amd as pm

    for name in _declared():
        assert hasattr(L, name), name
        assert name in pm.SIGNATURES, "binding lacks " + name


def test_status_strings(L):
    for st in range(7):
        assert L.pm_status_str(st)
    assert L.pm_status_str(0).decode() == "ok"


def test_host_validation_without_device(L):
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    # NULL pointers and zero lengths
    assert L.pm_poly_mul(null, 4, fake, 4, 998244353, fake, null) == 1
    assert L.pm_poly_mul(fake, 0, fake, 4, 998244353, fake, null) == 1
    # unsupported modulus
    assert L.pm_poly_mul(fake, 4, fake, 4, 1000000007, fake, null) == 2
    # transform length beyond the prime's 2-adic order (998244353: 2^23)
    assert L.pm_poly_mul(fake, 1 << 23, fake, 1 << 23, 998244353, fake, null) == 3
    assert L.pm_int_mul(fake, 1 << 23, fake, 1 << 23, fake, null) == 3
    assert L.pm_int_mul(null, 3, fake, 3, fake, null) == 1
    assert L.pm_int_mul_digits(fake, 3, fake, 3, 24, fake, null) == 1
    assert L.pm_int_mul_digits(fake, 1 << 23, fake, 1 << 23, 32, fake, null) == 3
    assert L.pm_ntt(fake, fake, 1, 998244353, 0, null) == 1           # n < 2
    assert L.pm_ntt(fake, fake, 3, 998244353, 0, null) == 2           # 3 does not divide p - 1
    assert L.pm_ntt(fake, fake, 18, 2013265921, 0, null) == 2         # odd part 9: no kernels
    assert L.pm_ntt(fake, fake, 3 << 25, 2013265921, 0, null) == 3    # 2^25 > 2^24
    assert L.pm_ntt(fake, fake, 7 << 24, 998244353, 0, null) == 3     # 2^24 > 2^23, the 2-adic order
    # general-radix product
    assert L.pm_poly_mul_mixed(null, 4, fake, 4, 2013265921, 3, fake, null) == 1
    assert L.pm_poly_mul_mixed(fake, 4, fake, 0, 2013265921, 3, fake, null) == 1
    assert L.pm_poly_mul_mixed(fake, 4, fake, 4, 998244353, 3, fake, null) == 2
    assert L.pm_poly_mul_mixed(fake, 4, fake, 4, 2013265921, 9, fake, null) == 2
    assert L.pm_poly_mul_mixed(fake, 4, fake, 4, 1000000007, 3, fake, null) == 2
    assert L.pm_poly_mul_mixed(fake, 7 << 23, fake, 7 << 23, 998244353, 7, fake, null) == 3
    assert L.pm_tft(fake, 5, 4, 2, 998244353, fake, null) == 1        # z > L
    assert L.pm_itft(fake, 1 << 10, 33, 998244353, fake, null) == 1   # n not a multiple of L/32
    assert L.pm_set_policy(7) == 1


def test_workspace_queries_on_host(L):
    """The queries need no device: sizes follow from the plans alone."""
    import paper_1609_01010_amd as pm

    n = ctypes.c_size_t(0)
    assert L.pm_workspace_query(1024, 1024, 998244353, ctypes.byref(n)) == 0 and n.value == 0  # one work-group
    assert L.pm_workspace_query(1 << 21, 1 << 21, 2013265921, ctypes.byref(n)) == 0
    assert n.value == 2 * 4 * (1 << 22)  # two operands of n' = L words
    for la, lb in ((600001, 400000), (70001, 9000), (40, 30)):
        assert L.pm_workspace_query(la, lb, 2013265921, ctypes.byref(n)) == 0
        P = pm.plan_for(la + lb - 1, 2013265921)
        want = 2 * 4 * (P.ma << (P.log_l - P.log_ra)) if P.kind == 2 else 0
        assert n.value == want, (la, lb, P)
    assert L.pm_workspace_query(4, 4, 1000000007, ctypes.byref(n)) == 2
    assert L.pm_workspace_query(0, 4, 998244353, ctypes.byref(n)) == 1
    assert L.pm_workspace_query(4, 4, 998244353, None) == 1
    assert L.pm_workspace_query(1 << 23, 1 << 23, 998244353, ctypes.byref(n)) == 3
    assert L.pm_int_mul_workspace_query(1 << 21, 1 << 21, ctypes.byref(n)) == 0
    assert n.value >= 3 * 4 * ((1 << 22) - 1) + 2 * (1 << 22)  # three residue arrays and the limb sums
    assert L.pm_int_mul_workspace_query(1 << 23, 1 << 23, ctypes.byref(n)) == 3
    # 32-bit digits halve the transforms: less workspace than the 16-bit limbs,
    # and the default choice at 2^21 + 2^21 limbs
    q = {}
    for d in (0, 16, 32):
        assert L.pm_int_mul_digits_workspace_query(1 << 21, 1 << 21, d, ctypes.byref(n)) == 0
        q[d] = n.value
    assert q[32] < q[16] and q[0] == q[32]
    assert q[32] >= 3 * 2 * 4 * (1 << 21) + 16 * ((1 << 21) - 1)  # three primes' Ta, Tb and the 16-byte x_k
    assert L.pm_int_mul_digits_workspace_query(1 << 21, 1 << 21, 8, ctypes.byref(n)) == 1
    # a batch needs the sum of its four-step items' workspaces (each rounded to 256 bytes)
    lens = [(100, 50), (5000, 4000), (70001, 9000), (300000, 20001), (40, 30)]
    probs = (pm.Problem * len(lens))()
    want = 0
    for i, (la, lb) in enumerate(lens):
        probs[i].a, probs[i].len_a, probs[i].b, probs[i].len_b = 4096, la, 4096, lb
        probs[i].p, probs[i].c = 998244353, 4096
        assert L.pm_workspace_query(la, lb, 998244353, ctypes.byref(n)) == 0
        want += (n.value + 255) // 256 * 256
    assert L.pm_batch_workspace_query(probs, len(lens), ctypes.byref(n)) == 0
    assert n.value == want and want > 0


def test_workspace_queries_bound_the_policies_without_a_device(L):
    """Under the learned policy the plan is chosen at call time (by the cost
    model on the device): the queries return the most any candidate needs,
    still on the host alone."""
    import paper_1609_01010_amd as pm

    n = ctypes.c_size_t(0)
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        assert L.pm_workspace_query(1 << 21, 1 << 21, 2013265921, ctypes.byref(n)) == 0
        assert n.value == 2 * 4 * (1 << 22)
        assert L.pm_workspace_query(600001, 400000, 2013265921, ctypes.byref(n)) == 0
        assert n.value == 2 * 4 * (1 << 20)  # a candidate without truncation
        assert L.pm_workspace_query(1024, 1024, 998244353, ctypes.byref(n)) == 0 and n.value == 0
        probs = (pm.Problem * 2)()
        for i, (la, lb) in enumerate(((600001, 400000), (1024, 1024))):
            probs[i].a, probs[i].len_a, probs[i].b, probs[i].len_b = 4096, la, 4096, lb
            probs[i].p, probs[i].c = 2013265921, 4096
        assert L.pm_batch_workspace_query(probs, 2, ctypes.byref(n)) == 0 and n.value == 2 * 4 * (1 << 20)
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)


def test_tuning_database_contexts_round_trip(tmp_path):
    """Rows of both timing contexts survive save and load; a row written
    without the context column loads as a single-product row."""
    import paper_1609_01010_amd as pm

    pm.tune_db_clear()
    P1 = pm.plan_candidates(70001, 998244353)[0]
    P2 = pm.plan_candidates(3000, 2013265921, general_radix=False)[-1]
    pm.tune_db_add(70001, 998244353, P1, 12.5, pm.CTX_SINGLE)
    pm.tune_db_add(3000, 2013265921, P2, 3.25, pm.CTX_BATCH)
    P3 = [P for P in pm.plan_candidates(70001, 998244353) if P.kind == pm.PLAN_MIXED][0]
    assert P3.q == 7
    pm.tune_db_add(70001, 998244353, P3, 9.75, pm.CTX_SINGLE)
    with pytest.raises(pm.PolymulError):
        pm.tune_db_add(70001, 998244353, P3, 9.75, pm.CTX_BATCH)  # products alone only
    path = str(tmp_path / "db.txt")
    pm.tune_db_save(path)
    pm.tune_db_clear()
    with open(path, "a") as f:
        # the 11-field line: no context (a single-product row), no odd factor
        f.write("70001 998244353 " + " ".join(str(v) for v in P1.as_tuple()[:8]) + " 11.0000\n")
    pm.tune_db_load(path)
    single, batch = pm.tune_db_rows(pm.CTX_SINGLE), pm.tune_db_rows(pm.CTX_BATCH)
    assert [(r[0], r[1], r[2].as_tuple(), r[3]) for r in single] == [(70001, 998244353, P1.as_tuple(), 12.5),
                                                                     (70001, 998244353, P3.as_tuple(), 9.75),
                                                                     (70001, 998244353, P1.as_tuple(), 11.0)]
    assert [(r[0], r[1], r[2].as_tuple(), r[3]) for r in batch] == [(3000, 2013265921, P2.as_tuple(), 3.25)]
    with pytest.raises(pm.PolymulError):
        pm.tune_db_add(3000, 2013265921, P2, 1.0, 7)  # no such context
    pm.tune_db_clear()


def test_features_carry_the_context():
    import paper_1609_01010_amd as pm

    P = pm.plan_candidates(70001, 998244353)[0]
    f0 = pm.model_features(70001, 998244353, P, pm.CTX_SINGLE)
    f1 = pm.model_features(70001, 998244353, P, pm.CTX_BATCH)
    assert f0.size == 17 and f0[16] == 0.0 and f1[16] == 1.0
    assert np.array_equal(f0[:16], f1[:16])


def test_general_radix_plans_stay_out_of_the_batch_and_the_model():
    """Kind-3 plans are for products alone: timing one in the batch context,
    its features and the model's prediction are refused before any device
    work."""
    import paper_1609_01010_amd as pm

    P = [Q for Q in pm.plan_candidates(40000, 2013265921) if Q.kind == pm.PLAN_MIXED][0]
    for call in (lambda: pm.time_plan(40000, 2013265921, P, reps=1, context=pm.CTX_BATCH),
                 lambda: pm.model_features(40000, 2013265921, P),
                 lambda: pm.model_predict(40000, 2013265921, [P])):
        with pytest.raises(pm.PolymulError) as e:
            call()
        assert e.value.status == pm.PM_EINVAL


def test_granularity(L):
    assert L.pm_itft_granularity(16) == 1
    assert L.pm_itft_granularity(32) == 1
    assert L.pm_itft_granularity(1 << 20) == 1 << 15


def test_plan_space_on_host():
    import paper_1609_01010_amd as pm

    for lc in (63, 64, 65, 2047, 5000, 40000, 1000000, (1 << 22) - 1):
        for p in pm.PRIMES:
            cands = pm.plan_candidates(lc, p)
            assert cands, (lc, p)
            pow2 = 1 << max(lc - 1, 1).bit_length()
            for P in cands:
                if P.kind == 0:
                    assert lc <= 64
                    continue
                if P.kind == 3:  # the shortest q 2^k >= lc, shorter than the power of two
                    assert (p - 1) % P.q == 0 and P.q in (3, 5, 7, 15, 17)
                    assert (P.q << (P.log_l - 1)) < lc <= (P.q << P.log_l) < pow2
                    continue
                nprime = P.ma << (P.log_l - P.log_ra)
                assert nprime >= lc
                assert 1 <= P.ma <= (1 << P.log_ra)
                if P.kind == 2:
                    assert P.log_l == P.log_ra + P.log_rb + P.log_c
    # the general-radix plans, last, for the odd factors of p - 1
    mixed = [(P.q, P.log_l) for P in pm.plan_candidates(40000, 2013265921) if P.kind == 3]
    assert mixed == [(3, 14), (5, 13), (15, 12)]  # 49152, 40960, 61440 < 65536
    assert [P.q for P in pm.plan_candidates(40000, 998244353) if P.kind == 3] == [7]  # 57344 (17: 69632)
    assert all(P.kind != 3 for P in pm.plan_candidates(40000, 998244353, general_radix=False))
    assert not [P for P in pm.plan_candidates(1 << 15, 2013265921) if P.kind == 3]
    # truncation: a length just past a power of two is not padded to 2L
    P = pm.plan_for(1000000, 2013265921)
    assert (P.ma << (P.log_l - P.log_ra)) < (1 << 20)
    P = pm.plan_for(2047, 998244353)
    assert P.kind == 1 and P.log_l == 11


_ENV_CHILD = r"""
import os, sys
import numpy as np
import paper_1609_01010_amd as pm

db, weights = sys.argv[1], sys.argv[2]
assert pm.get_policy() == pm.POLICY_DEFAULT
P1 = pm.plan_candidates(70001, 998244353)[0]
P2 = pm.plan_candidates(3000, 2013265921, general_radix=False)[-1]
pm.tune_db_add(70001, 998244353, P1, 12.5, pm.CTX_SINGLE)
pm.tune_db_add(3000, 2013265921, P2, 3.25, pm.CTX_BATCH)
pm.tune_db_save(db)
pm.tune_db_clear()

def status(f):
    try:
        f()
        return 0
    except pm.PolymulError as e:
        return e.status

# empty variables change nothing
os.environ.update(PM_PLAN_POLICY="", PM_TUNE_DB="", PM_MLP_WEIGHTS="")
pm.config_from_env()
assert pm.get_policy() == pm.POLICY_DEFAULT and pm.lib().pm_tune_db_size() == 0
assert status(pm.model_get) != 0  # no model yet

# an unknown policy name is refused before the files are read
os.environ.update(PM_PLAN_POLICY="fastest", PM_TUNE_DB=db, PM_MLP_WEIGHTS=weights)
assert status(pm.config_from_env) == pm.PM_EINVAL
assert pm.get_policy() == pm.POLICY_DEFAULT and pm.lib().pm_tune_db_size() == 0
assert status(pm.model_get) != 0

# a missing database: the error is returned and the policy is not set
os.environ.update(PM_PLAN_POLICY="exhaustive", PM_TUNE_DB=db + ".missing")
assert status(pm.config_from_env) == pm.PM_EINVAL
assert pm.get_policy() == pm.POLICY_DEFAULT

# all three applied
os.environ.update(PM_PLAN_POLICY="learned", PM_TUNE_DB=db)
pm.config_from_env()
assert pm.get_policy() == pm.POLICY_LEARNED
rows = [(r[0], r[1], r[2].as_tuple(), r[3]) for r in pm.tune_db_rows(pm.CTX_SINGLE)]
assert rows == [(70001, 998244353, P1.as_tuple(), 12.5)], rows
rows = [(r[0], r[1], r[2].as_tuple(), r[3]) for r in pm.tune_db_rows(pm.CTX_BATCH)]
assert rows == [(3000, 2013265921, P2.as_tuple(), 3.25)], rows
w, mean, sd = pm.model_get()
vals = open(weights).read().split("\n")
assert (mean, sd) == tuple(float(np.float32(v)) for v in vals[1].split()), (mean, sd)
want = np.array([float(v) for v in vals[2:] if v.strip()], dtype=np.float32)
assert np.array_equal(w, want)

# the other names set the policy too
for name, want_policy in (("exhaustive", pm.POLICY_EXHAUSTIVE), ("default", pm.POLICY_DEFAULT)):
    os.environ.update(PM_PLAN_POLICY=name, PM_TUNE_DB="", PM_MLP_WEIGHTS="")
    pm.config_from_env()
    assert pm.get_policy() == want_policy
print("env ok")
"""


def test_plan_choice_from_the_environment(tmp_path):
    """PM_PLAN_POLICY, PM_TUNE_DB and PM_MLP_WEIGHTS are applied on the host
    (in a child process, so the loaded model stays out of this one): empty
    variables change nothing, an unknown policy name and a missing file are
    refused without setting the policy, and the database rows and the weights
    arrive exactly as written."""
    import subprocess
    import sys

    weights = os.path.join(ROOT, "paper_1609_01010_amd", "data", "cost_model.txt")
    env = {k: v for k, v in os.environ.items() if not k.startswith("PM_")}
    r = subprocess.run([sys.executable, "-c", _ENV_CHILD, str(tmp_path / "db.txt"), weights], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "env ok" in r.stdout, r.stdout + r.stderr
