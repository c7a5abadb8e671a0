"""Learned plan selection, end to end on one GPU.

1. The tuner times every candidate plan of each training length (every power
   of two 2^10..2^20 plus 300 non-power-of-two lengths log-uniform in
   [2^10, 2^20]) and records the timing database.
2. The cost model is trained on those rows by the library's own kernels.
3. On the held-out lengths (2^21..2^24 plus 200 non-power-of-two lengths
   log-uniform in [2^10, 2^24]) the model's pick is compared with the fastest
   plan found by timing every candidate (exhaustive search), and with the
   default plan (the library without the model).

Regret of a length = t(pick) / t(best) - 1.  The exhaustive pass takes the
median of `reps` runs per candidate; the minimum over many noisy candidates
is biased low, so the pick, the best and the default plan are then re-timed
interleaved (three rounds of `reps` runs each, median of the three medians)
and the regret is computed from those.  Reported: the geometric mean of
(1 + regret) - 1 over the held-out set, the maximum, the fraction at or below
5%, and the gain of the learned policy over the default one (geometric mean
of t(default) / t(pick)).  All products use p = 2013265921 (transforms up to
2^27 exist for it).

    python -m paper_1609_01010_amd.learned_eval --out DIR [--reps 5] [--quick]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs

P = 2013265921


def log(*a):
    print(*a, flush=True)


def geomean(xs):
    xs = np.asarray(xs, dtype=np.float64)
    return float(np.exp(np.mean(np.log(xs))))


def run(out_dir: str, reps: int = 5, steps: int = 3000, lr: float = 3e-3, quick: bool = False):
    import paper_1609_01010_amd as pm

    os.makedirs(out_dir, exist_ok=True)
    pm.lib()
    pm.tune_db_clear()
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_DEFAULT)
    n_train_rnd, n_held_rnd = (30, 20) if quick else (300, 200)
    train = inputs.tuning_lengths(n_random=n_train_rnd)
    held = inputs.heldout_lengths(n_random=n_held_rnd, exclude=train)
    t0 = time.time()
    for i in range(0, len(train), 16):
        pm.tune(train[i:i + 16], P, reps=reps)
        log(f"tuned {min(i + 16, len(train))}/{len(train)} training lengths ({time.time() - t0:.0f} s)")
    pm.tune_db_save(os.path.join(out_dir, "tuning_db.txt"))
    rows = pm.tune_db_rows()
    losses = pm.model_train(inputs.mlp_init(), steps=steps, lr=lr)
    log(f"trained on {len(rows)} rows: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    pm.model_save(os.path.join(out_dir, "cost_model.txt"))

    recs = []
    for k, lc in enumerate(held):
        cands = pm.plan_candidates(lc, P)
        pred = pm.model_predict(lc, P, cands)
        pick = cands[int(np.argmin(pred))]
        default = pm.plan_for(lc, P)  # the default policy (nothing cached for held-out lengths)
        times = [pm.time_plan(lc, P, Q, reps=reps) for Q in cands]
        best = int(np.argmin(times))
        trio = {"pick": pick, "best": cands[best], "default": default}
        rt = {k: [] for k in trio}
        for _ in range(3):
            for name, Q in trio.items():
                rt[name].append(pm.time_plan(lc, P, Q, reps=reps))
        t_pick, t_best, t_def = (float(np.median(rt[name])) for name in ("pick", "best", "default"))
        recs.append({
            "lc": lc, "candidates": len(cands), "t_best_us": t_best, "t_pick_us": t_pick,
            "t_default_us": t_def, "regret": max(t_pick / t_best - 1.0, 0.0),
            "regret_first_pass": times[int(np.argmin(pred))] / times[best] - 1.0,
            "best": list(cands[best].as_tuple()), "pick": list(pick.as_tuple()),
            "pred_err_log": float(pred[int(np.argmin(pred))] - math.log(t_pick)),
        })
        if k % 10 == 0 or k < 4:
            log(f"held-out {k + 1}/{len(held)} lc={lc}: regret {recs[-1]['regret']:.3f} "
                f"best {times[best]:.1f} us pick {t_pick:.1f} us default {t_def:.1f} us")
    reg = [r["regret"] for r in recs]
    summary = {
        "prime": P,
        "train_lengths": len(train),
        "train_rows": len(rows),
        "heldout_lengths": len(held),
        "loss_first": float(losses[0]),
        "loss_last": float(losses[-1]),
        "regret_geomean": geomean([1 + r for r in reg]) - 1,
        "regret_max": float(max(reg)),
        "regret_frac_le_5pct": float(np.mean([r <= 0.05 for r in reg])),
        "gain_vs_default_geomean": geomean([r["t_default_us"] / r["t_pick_us"] for r in recs]),
        "default_regret_geomean": geomean([max(r["t_default_us"] / r["t_best_us"], 1.0) for r in recs]) - 1,
        "regret_first_pass_geomean": geomean([1 + max(r["regret_first_pass"], 0.0) for r in recs]) - 1,
        "pow2_heldout": [r for r in recs if r["lc"] & (r["lc"] - 1) == 0],
        "wall_s": time.time() - t0,
    }
    with open(os.path.join(out_dir, "learned_eval.json"), "w") as f:
        json.dump({"summary": summary, "heldout": recs}, f, indent=1)
    log(json.dumps({k: v for k, v in summary.items() if k != "pow2_heldout"}))
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--quick", action="store_true", help="30 + 20 random lengths instead of 300 + 200")
    a = ap.parse_args(argv)
    run(a.out, reps=a.reps, steps=a.steps, quick=a.quick)


if __name__ == "__main__":
    sys.exit(main())
