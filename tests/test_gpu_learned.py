"""The tuner and the learned cost model on the GPU.

The network's forward, backward and Adam kernels run in float32 and are
checked against the oracle's float64 network (oracle/mlp.py) with a relative
tolerance of 1e-4 per tensor (largest absolute difference over the largest
reference magnitude): float32 accumulation over at most 64-term dot products
and a 32-sample batch stays far inside that.
"""

import sys

import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import poly as op
from paper_1609_01010_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(B=32, tag=8):
    rng = inputs.rng_for(tag)
    X = rng.uniform(-1, 1, (B, inputs.MLP_F)).astype(np.float32)
    t = rng.normal(0, 1, B).astype(np.float32)
    return X, t


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


def test_mlp_forward_and_gradients_match_oracle(gpu_lib):
    pm = gpu_lib
    w = inputs.mlp_init()
    X, t = _batch()
    P = inputs.mlp_unflatten(w)
    y_ref, _ = omlp.forward(P, X)
    y = pm.mlp_forward(w, X)
    assert _rel(y, y_ref) <= TOL
    loss, g = pm.mlp_loss_grad(w, X, t)
    assert abs(loss - omlp.loss(P, X, t)) <= TOL * abs(omlp.loss(P, X, t))
    g_ref = omlp.backward(P, X, t)
    G = inputs.mlp_unflatten(g)
    for k in omlp.NAMES:
        say("grad", k, _rel(G[k], g_ref[k]))
        assert _rel(G[k], g_ref[k]) <= TOL, k


def test_mlp_adam_matches_oracle(gpu_lib):
    pm = gpu_lib
    w = inputs.mlp_init()
    X, t = _batch()
    _, g = pm.mlp_loss_grad(w, X, t)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    P = inputs.mlp_unflatten(w)
    G = inputs.mlp_unflatten(g)
    state = {}
    ref = {k: np.array(P[k]) for k in omlp.NAMES}
    for step in (1, 2, 3):
        w, m, v = pm.mlp_adam(w, g, m, v, step, 1e-3)
        omlp.adam_step(ref, G, state, lr=1e-3)
    W = inputs.mlp_unflatten(w)
    for k in omlp.NAMES:
        assert _rel(W[k], ref[k]) <= TOL, k


def test_mlp_training_follows_oracle_and_learns(gpu_lib):
    pm = gpu_lib
    w0 = inputs.mlp_init()
    rng = inputs.rng_for(9)
    X = rng.uniform(-1, 1, (64, inputs.MLP_F)).astype(np.float32)
    t = (np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    w, losses = pm.mlp_train(w0, X, t, steps=5, lr=1e-3)
    ref = omlp.train(inputs.mlp_unflatten(w0), X, t, steps=5, lr=1e-3)
    W = inputs.mlp_unflatten(w)
    for k in omlp.NAMES:
        say("trajectory", k, _rel(W[k], ref[k]))
        assert _rel(W[k], ref[k]) <= TOL, k
    w, losses = pm.mlp_train(w0, X, t, steps=400, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0]


def test_tuner_records_every_candidate_and_caches_the_best(gpu_lib):
    pm = gpu_lib
    p = 998244353
    pm.tune_db_clear()
    pm.plan_cache_clear()
    lcs = [3000, 70001]
    pm.tune(lcs, p, reps=3)
    rows = pm.tune_db_rows()
    for lc in lcs:
        mine = [r for r in rows if r[0] == lc]
        assert len(mine) == len(pm.plan_candidates(lc, p))
        assert all(r[3] > 0 for r in mine)
        best = min(mine, key=lambda r: r[3])[2]
        assert pm.plan_for(lc, p).as_tuple() == best.as_tuple()
        la, lb = inputs.split_output_length(lc)
        a, b = inputs.poly_pair((110, lc), la, lb, p)
        import torch

        c = pm.poly_mul(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), p)
        assert np.array_equal(c.cpu().numpy(), op.poly_mul(a, b, p))
    pm.plan_cache_clear()


def test_batch_context_tuning_drives_the_batch(gpu_lib):
    """Tuning in the batch context times each candidate as a batch of
    products (rows recorded with that context, the best in the batch
    context's cache); pm_poly_mul_batch then runs those plans, exactly."""
    import torch

    pm = gpu_lib
    p = 998244353
    pm.tune_db_clear()
    pm.plan_cache_clear()
    lcs = [3000, 70001]
    pm.tune(lcs, p, reps=3, context=pm.CTX_BATCH)
    assert pm.tune_db_rows(pm.CTX_SINGLE) == []
    rows = pm.tune_db_rows(pm.CTX_BATCH)
    for lc in lcs:
        mine = [r for r in rows if r[0] == lc]
        assert len(mine) == len(pm.plan_candidates(lc, p, general_radix=False)) and all(r[3] > 0 for r in mine)
        best = min(mine, key=lambda r: r[3])[2]
        # per-product time of the best plan, timed again in the batch context
        assert pm.time_plan(lc, p, best, reps=3, context=pm.CTX_BATCH) > 0
    items = []
    for k in range(6):
        for lc in lcs:
            la, lb = inputs.split_output_length(lc)
            items.append(inputs.poly_pair((112, lc, k), la, lb, p))
    outs = pm.poly_mul_batch([(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), p) for a, b in items])
    assert pm.stream_check() == 0
    for (a, b), c in zip(items, outs):
        assert np.array_equal(c.cpu().numpy(), op.poly_mul(a, b, p))
    pm.tune_db_clear()
    pm.plan_cache_clear()


def test_learned_batch_policy_stays_exact(gpu_lib):
    """The shipped cost model under the learned policy on a batch of uneven
    products: the first call plans the batch per size class and compares the
    whole batch with the default plans; later calls of the same shape (new
    operand and output buffers) take the repeated-shape path.  Every product
    of every call is exact, and the batch context's plans are valid plans of
    the candidate space."""
    import os

    import torch

    pm = gpu_lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))
    items = inputs.batch_uneven(count=96, lo=16, hi=40000, tag=(113,))
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        for rnd in range(3):
            probs = [(torch.from_numpy(it.a).cuda(), torch.from_numpy(it.b).cuda(), it.p) for it in items]
            say("case: learned batch, call", rnd)
            outs = pm.poly_mul_batch(probs)
            assert pm.stream_check() == 0
            for it, c in zip(items, outs):
                assert np.array_equal(c.cpu().numpy(), op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p]))
        for it in items[:12]:
            lc = it.a.size + it.b.size - 1
            P = pm.plan_for(lc, it.p, pm.CTX_BATCH)
            assert any(P.as_tuple() == Q.as_tuple() for Q in pm.plan_candidates(lc, it.p)), (lc, P)
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)
        pm.plan_cache_clear()


def test_learned_policy_integer_product_in_caller_workspace(gpu_lib):
    """Under the learned policy the integer product's plans come from the cost
    model at call time, so its workspace query returns the most any candidate
    plan and digit size could need: a caller workspace of exactly that size
    runs the product (whatever digits the model's plans allow), exact against
    CPython, and so does one sized for forced 16-bit digits."""
    import os

    import torch

    pm = gpu_lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))
    rng = np.random.default_rng(117)
    s = torch.cuda.Stream()
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        for na, nb in ((5000, 3001), (100001, 77777), (1 << 18, (1 << 18) - 3)):
            a = rng.integers(0, 1 << 16, na, dtype=np.uint16)
            b = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
            want = op.int_mul(a, b)
            for digits in (None, 16):
                need = pm.int_mul_workspace_query(na, nb, digits=digits)
                say("case: learned int product in a caller workspace", na, nb, digits, need)
                buf = torch.empty(need, dtype=torch.uint8, device="cuda")
                torch.cuda.synchronize()
                pm.set_workspace(buf, stream=s)
                try:
                    with torch.cuda.stream(s):
                        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
                        c = pm.int_mul(ta, tb, stream=s, digits=digits)
                    s.synchronize()
                finally:
                    pm.set_workspace(None, stream=s)
                assert pm.stream_check() == 0
                assert np.array_equal(c.cpu().numpy(), want), (na, nb, digits)
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)
        pm.plan_cache_clear()


def test_learned_policy_trains_predicts_and_stays_exact(gpu_lib, tmp_path):
    """A small version of the learned-plan experiment: tune a few lengths,
    train the network on the device, pick plans for unseen lengths; the
    products stay bit-exact and the pick is never far from the tuned best."""
    import torch

    pm = gpu_lib
    p = 2013265921
    pm.tune_db_clear()
    pm.plan_cache_clear()
    train = [1 << k for k in range(10, 18)] + [1500, 3001, 9000, 23000, 50001, 100003]
    pm.tune(train, p, reps=3)
    losses = pm.model_train(inputs.mlp_init(), steps=1500, lr=3e-3)
    say("loss", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
    # save and load round trip
    path = str(tmp_path / "model.txt")
    pm.model_save(path)
    w, mean, sd = pm.model_get()
    pm.model_load(path)
    w2, mean2, sd2 = pm.model_get()
    assert np.array_equal(w, w2) and mean == mean2 and sd == sd2
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        for lc in (5000, 40000, 150001):
            P = pm.plan_for(lc, p)
            cands = pm.plan_candidates(lc, p, general_radix=False)
            pred = pm.model_predict(lc, p, cands)
            assert P.as_tuple() == cands[int(np.argmin(pred))].as_tuple()
            la, lb = inputs.split_output_length(lc)
            a, b = inputs.poly_pair((111, lc), la, lb, p)
            c = pm.poly_mul(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), p)
            assert np.array_equal(c.cpu().numpy(), op.poly_mul(a, b, p))
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)
        pm.plan_cache_clear()


def test_learned_batch_policy_keeps_the_faster_plans(gpu_lib):
    """The first call of a batch shape under the learned policy runs the
    batch with the model's plans and with the default plans and keeps the
    faster.  A model whose output is negated picks, per size class, the plan
    family it predicts slowest, so the default plans must be kept, also by
    the later calls of the shape (the repeated-shape path); every product of
    every call is exact."""
    import os

    import torch

    pm = gpu_lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))
    w, mean, sd = pm.model_get()
    w[-(inputs.MLP_H + 1):] *= -1.0  # the output layer: predictions negated
    items = inputs.batch_uneven(count=128, lo=64, hi=20000, tag=(114,))
    lcs = [it.a.size + it.b.size - 1 for it in items]
    pm.set_policy(pm.POLICY_DEFAULT)
    pm.plan_cache_clear()
    default = [pm.plan_for(lc, it.p, pm.CTX_BATCH).as_tuple() for lc, it in zip(lcs, items)]
    pm.model_set(w, mean, sd)
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        for rnd in range(2):
            probs = [(torch.from_numpy(it.a).cuda(), torch.from_numpy(it.b).cuda(), it.p) for it in items]
            say("case: learned batch with a negated model, call", rnd)
            outs = pm.poly_mul_batch(probs)
            assert pm.stream_check() == 0
            used = [P.as_tuple() for P in pm.batch_plans_used(len(items))]
            assert used == default, rnd
            for it, c in zip(items, outs):
                assert np.array_equal(c.cpu().numpy(), op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p]))
        # the comparison was real: the negated model's plans (now in the batch
        # context's plan cache) differ from the default ones
        model = [pm.plan_for(lc, it.p, pm.CTX_BATCH).as_tuple() for lc, it in zip(lcs, items)]
        assert sum(m != d for m, d in zip(model, default)) >= len(items) // 4
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)
        pm.plan_cache_clear()
        pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))


def test_learned_plans_on_the_4096_product_batch(gpu_lib):
    """The launch configuration bench.py times: the 4096 uneven products under
    the learned policy with the shipped cost model (batch context, plans
    checked against the default ones on the first call), then the repeated
    shape on a second buffer set; every product of both calls against the
    oracle's transform route."""
    import os

    import torch

    pm = gpu_lib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))
    items = inputs.batch_uneven()
    want = [op.poly_mul_ntt(it.a, it.b, it.p, inputs.PRIMES[it.p]) for it in items]
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_LEARNED)
    try:
        for call in range(2):
            probs = [(torch.from_numpy(it.a).cuda(), torch.from_numpy(it.b).cuda(), it.p) for it in items]
            say("case: learned 4096-product batch, call", call)
            outs = pm.poly_mul_batch(probs)
            assert pm.stream_check() == 0
            for k, (w, c) in enumerate(zip(want, outs)):
                assert np.array_equal(c.cpu().numpy(), w), (call, k)
        used = pm.batch_plans_used(len(items))
        assert sum(P.kind == 2 for P in used) > len(items) // 2
    finally:
        pm.set_policy(pm.POLICY_DEFAULT)
        pm.plan_cache_clear()


def _geomean(xs):
    return float(np.exp(np.mean(np.log(np.asarray(xs, dtype=np.float64)))))


def test_shipped_model_regret_and_gain_on_heldout_lengths(gpu_lib):
    """The shipped cost model (trained on the autotuner's timings of the
    powers of two 2^10..2^20 and of non-powers of two up to 2^23, none of
    them held out) on 16 held-out lengths: 2^21, 2^22 and 14
    non-powers of two log-uniform in [2^10, 2^24], mod 2013265921, products
    on their own.  Per length every candidate plan is timed (the exhaustive
    search); the model's pick, that best plan and the default plan (the
    library without the model) are then re-timed interleaved, three rounds of
    five runs, median.  Regret = t(pick) / t(best) - 1.  Asserts the
    geometric-mean regret is at most 5% and that the model's picks beat the
    default plans (geometric mean of t(default) / t(pick) above 1)."""
    import os

    pm = gpu_lib
    p = 2013265921
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pm.model_load(os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt"))
    held = inputs.heldout_lengths(n_random=200, exclude=inputs.tuning_lengths())
    lengths = [1 << 21, 1 << 22] + held[4:18]
    regrets, gains = [], []
    pm.set_policy(pm.POLICY_DEFAULT)
    try:
        for lc in lengths:
            pm.plan_cache_clear()
            cands = pm.plan_candidates(lc, p, general_radix=False)
            pick = cands[int(np.argmin(pm.model_predict(lc, p, cands)))]
            default = pm.plan_for(lc, p)
            pm.tune_db_clear()
            pm.tune([lc], p, reps=5)
            # the best of the model's space (the power-of-two plans)
            rows = [r for r in pm.tune_db_rows() if r[0] == lc and r[1] == p and r[2].kind != pm.PLAN_MIXED]
            assert len(rows) == len(cands)
            best = min(rows, key=lambda r: r[3])[2]
            t = {"pick": [], "best": [], "default": []}
            for _ in range(3):
                for name, plan in (("pick", pick), ("best", best), ("default", default)):
                    t[name].append(pm.time_plan(lc, p, plan, reps=5))
            tp, tb, td = (float(np.median(t[k])) for k in ("pick", "best", "default"))
            regrets.append(max(tp / tb - 1.0, 0.0))
            gains.append(td / tp)
            say(f"lc={lc}: best {tb:.1f} us, pick {tp:.1f} us, default {td:.1f} us, regret {regrets[-1]:.3f}")
    finally:
        pm.tune_db_clear()
        pm.plan_cache_clear()
    reg = _geomean([1 + r for r in regrets]) - 1
    gain = _geomean(gains)
    say(f"geometric-mean regret {reg:.4f}, max {max(regrets):.3f}, gain over the default plans {gain:.3f}")
    assert reg <= 0.05
    assert gain > 1.0


_INIT_ENV_CHILD = r"""
import sys
import numpy as np
import torch
import paper_1609_01010_amd as pm
from oracle import poly as op
from paper_1609_01010_amd import inputs

mode = sys.argv[1]
if mode == "bad":
    try:
        pm.init()
    except pm.PolymulError as e:
        assert e.status == pm.PM_EINVAL
        try:
            pm.init()  # refused again: the environment is read once, its status kept
        except pm.PolymulError as e2:
            assert e2.status == pm.PM_EINVAL
            assert pm.get_policy() == pm.POLICY_DEFAULT
            print("init env ok", flush=True)
            sys.exit(0)
    sys.exit("a bad PM_PLAN_POLICY was not refused")
pm.init()
assert pm.get_policy() == pm.POLICY_LEARNED
p = 998244353
a, b = inputs.poly_pair(31, 30001, 20001, p)
c = pm.poly_mul(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), p)
assert pm.stream_check() == 0
assert np.array_equal(c.cpu().numpy(), op.poly_mul(a, b, p))
print("init env ok", flush=True)
"""


@pytest.mark.parametrize("mode", ["learned", "bad"])
def test_init_applies_the_environment(mode, tmp_path):
    """The first pm_init of a process applies PM_PLAN_POLICY and
    PM_MLP_WEIGHTS: under 'learned' with the shipped weights the policy is in
    force and a product matches the oracle exactly; an unknown policy name
    makes pm_init fail with PM_EINVAL, every time, and sets nothing."""
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = {k: v for k, v in os.environ.items() if not k.startswith("PM_")}
    env["PM_PLAN_POLICY"] = "learned" if mode == "learned" else "quickest"
    env["PM_MLP_WEIGHTS"] = os.path.join(root, "paper_1609_01010_amd", "data", "cost_model.txt")
    say("child pm_init with PM_PLAN_POLICY=" + env["PM_PLAN_POLICY"])
    r = subprocess.run([sys.executable, "-c", _INIT_ENV_CHILD, mode], cwd=root, env=env, capture_output=True,
                       text=True, timeout=100)
    assert r.returncode == 0 and "init env ok" in r.stdout, r.stdout + r.stderr
