"""Learned plan selection, end to end on one GPU.

1. The tuner times every candidate plan of each training length (every power
   of two 2^10..2^20, 300 non-power-of-two lengths log-uniform in
   [2^10, 2^20] and 60 in [2^20, 2^23]), for each of the four primes, in
   both timing contexts: a
   product on its own, and the time per product of a batch of about 2^24 / L
   products of the length (enough to keep the device full).
2. The cost model is trained on all those rows by the library's own kernels;
   the context is one of its features.
3. On the held-out lengths (2^21..2^24 plus 200 non-power-of-two lengths
   log-uniform in [2^10, 2^24]), in each context, the model's pick is
   compared with the fastest plan found by timing every candidate (exhaustive
   search), and with the default plan (the library without the model).
4. The 4096-product batch is timed with the default plans, with the model's
   picks for the batch context (what the batch executor uses), and with the
   model's picks for products on their own forced onto the batch.

Regret of a length = t(pick) / t(best) - 1.  The exhaustive pass takes the
median of `reps` runs per candidate; the minimum over many noisy candidates
is biased low, so the pick, the best and the default plan are then re-timed
interleaved (three rounds of `reps` runs each, median of the three medians)
and the regret is computed from those.  Reported per context: the geometric
mean of (1 + regret) - 1 over the held-out set, the maximum, the fraction at
or below 5%, and the gain of the learned policy over the default one
(geometric mean of t(default) / t(pick)).  The held-out products of step 3
use p = 2013265921 (transforms up to 2^27 exist for it).

    python -m paper_1609_01010_amd.learned_eval --out DIR [--reps 5] [--quick]
    python -m paper_1609_01010_amd.learned_eval --out DIR --batch-families

With --model PATH, steps 1 and 2 are skipped and the given cost model (for
instance the shipped data/cost_model.txt) is evaluated.  With --budget S the
held-out loop stops after about S seconds and keeps what it measured in
DIR/heldout_partial.json; run the same command again to resume (exit status
3 while incomplete).
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


def run(out_dir: str, reps: int = 5, steps: int = 3000, lr: float = 3e-3, quick: bool = False,
        model: str | None = None, budget: float | None = None):
    import torch

    import paper_1609_01010_amd as pm

    torch.zeros(1, device="cuda")  # torch takes the device before the library does (the batch step uses both)

    os.makedirs(out_dir, exist_ok=True)
    pm.lib()
    pm.tune_db_clear()
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_DEFAULT)
    n_train_rnd, n_held_rnd = (30, 20) if quick else (300, 200)
    train = inputs.tuning_lengths(n_random=n_train_rnd, n_large=6 if quick else 60)
    held = inputs.heldout_lengths(n_random=n_held_rnd, exclude=train)
    t0 = time.time()
    if model:
        pm.model_load(model)
        n_rows = {pm.CTX_SINGLE: None, pm.CTX_BATCH: None}
        losses = [float("nan")]
    else:
        for ctx, cname in ((pm.CTX_SINGLE, "single"), (pm.CTX_BATCH, "batch")):
            for q in inputs.PRIME_LIST:
                for i in range(0, len(train), 32):
                    pm.tune(train[i:i + 32], q, reps=reps, context=ctx)
                log(f"tuned {len(train)} training lengths mod {q}, {cname} ({time.time() - t0:.0f} s)")
        pm.plan_cache_clear()
        pm.tune_db_save(os.path.join(out_dir, "tuning_db.txt"))
        n_rows = {c: len(pm.tune_db_rows(c)) for c in (pm.CTX_SINGLE, pm.CTX_BATCH)}
        losses = pm.model_train(inputs.mlp_init(), steps=steps, lr=lr)
        log(f"trained on {sum(n_rows.values())} rows: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
        pm.model_save(os.path.join(out_dir, "cost_model.txt"))

    partial = os.path.join(out_dir, "heldout_partial.json")
    recs = {"single": [], "batch": []}
    if model and os.path.exists(partial):
        with open(partial) as f:
            recs = json.load(f)
        log(f"resuming: {len(recs['single'])} + {len(recs['batch'])} held-out records")
    for ctx, cname in ((pm.CTX_SINGLE, "single"), (pm.CTX_BATCH, "batch")):
        done = {r["lc"] for r in recs[cname]}
        for k, lc in enumerate(held):
            if lc in done:
                continue
            if budget is not None and time.time() - t0 > budget:
                with open(partial, "w") as f:
                    json.dump(recs, f)
                log(f"budget spent: {len(recs['single'])} + {len(recs['batch'])} of {2 * len(held)} held-out records")
                return None
            cands = pm.plan_candidates(lc, P, general_radix=False)
            pred = pm.model_predict(lc, P, cands, context=ctx)
            ipick = int(np.argmin(pred))
            pick = cands[ipick]
            default = pm.plan_for(lc, P)  # the default policy (nothing cached for held-out lengths)
            pm.tune_db_clear()
            pm.tune([lc], P, reps=reps, context=ctx)
            timed = {tuple(Q.as_tuple()): us for (_, _, Q, us) in pm.tune_db_rows(ctx)}
            pm.plan_cache_clear()
            times = [timed[tuple(Q.as_tuple())] for Q in cands]
            best = int(np.argmin(times))
            trio = {"pick": pick, "best": cands[best], "default": default}
            rt = {name: [] for name in trio}
            for _ in range(3):
                for name, Q in trio.items():
                    rt[name].append(pm.time_plan(lc, P, Q, reps=reps, context=ctx))
            t_pick, t_best, t_def = (float(np.median(rt[name])) for name in ("pick", "best", "default"))
            recs[cname].append({
                "lc": lc, "candidates": len(cands), "t_best_us": t_best, "t_pick_us": t_pick,
                "t_default_us": t_def, "regret": max(t_pick / t_best - 1.0, 0.0),
                "regret_first_pass": times[ipick] / times[best] - 1.0,
                "best": list(cands[best].as_tuple()), "pick": list(pick.as_tuple()),
                "pred_err_log": float(pred[ipick] - math.log(t_pick)),
            })
            if budget is not None:
                with open(partial, "w") as f:
                    json.dump(recs, f)
            if k % 20 == 0 or k < 2:
                r = recs[cname][-1]
                log(f"held-out {cname} {k + 1}/{len(held)} lc={lc}: regret {r['regret']:.3f} "
                    f"best {times[best]:.1f} us pick {t_pick:.1f} us default {t_def:.1f} us")
    pm.tune_db_clear()

    def ctx_summary(rs):
        reg = [r["regret"] for r in rs]
        return {
            "regret_geomean": geomean([1 + r for r in reg]) - 1,
            "regret_max": float(max(reg)),
            "regret_frac_le_5pct": float(np.mean([r <= 0.05 for r in reg])),
            "gain_vs_default_geomean": geomean([r["t_default_us"] / r["t_pick_us"] for r in rs]),
            "default_regret_geomean": geomean([max(r["t_default_us"] / r["t_best_us"], 1.0) for r in rs]) - 1,
            "regret_first_pass_geomean": geomean([1 + max(r["regret_first_pass"], 0.0) for r in rs]) - 1,
        }

    single = ctx_summary(recs["single"])
    summary = {
        "prime": P,
        "train_lengths": len(train),
        "train_rows": n_rows[pm.CTX_SINGLE],
        "train_rows_batch": n_rows[pm.CTX_BATCH],
        "heldout_lengths": len(held),
        "loss_first": float(losses[0]),
        "loss_last": float(losses[-1]),
        **single,
        "batch_context": ctx_summary(recs["batch"]),
        "uneven_batch_4096": batch_policies(pm, reps),
        "wall_s": time.time() - t0,
    }
    with open(os.path.join(out_dir, "learned_eval.json"), "w") as f:
        json.dump({"summary": summary, "heldout": recs["single"], "heldout_batch": recs["batch"]}, f, indent=1)
    log(json.dumps(summary))
    return summary


def batch_policies(pm, reps: int):
    """The 4096 uneven products (four primes) as one batch, with three plan
    choices: the default plans, the model's picks for the batch context (what
    pm_poly_mul_batch uses under the learned policy), and the model's picks for
    products on their own forced onto the batch (plan cache)."""
    import torch

    items = inputs.batch_uneven()
    dev = torch.device("cuda")
    probs = [(torch.from_numpy(it.a).to(dev), torch.from_numpy(it.b).to(dev), it.p) for it in items]
    outs = [torch.empty(it.a.size + it.b.size - 1, dtype=torch.uint32, device=dev) for it in items]

    def timed():
        pb = pm.PreparedBatch(probs, outs=outs)
        pb.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(7, reps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pb.run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {}
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_DEFAULT)
    out["default_ms"] = timed()
    pm.set_policy(pm.POLICY_LEARNED)
    pm.plan_cache_clear()
    out["learned_batch_context_ms"] = timed()
    pm.plan_cache_clear()
    for it in items:
        lc = it.a.size + it.b.size - 1
        if lc > 64:
            pm.plan_cache_put(lc, it.p, pm.plan_for(lc, it.p))  # the single-context pick
    out["learned_single_context_ms"] = timed()
    pm.plan_cache_clear()
    pm.set_policy(pm.POLICY_DEFAULT)
    if pm.stream_check() != 0:
        raise SystemExit("device error in the batch")
    log(f"4096 uneven products: {json.dumps(out)}")
    return out


def batch_families(pm, model: str, out_dir: str, n_classes: int = 3, k: int = 30):
    """The learned batch plans against a search on the whole batch: the 4096
    uneven products run with the model's plans (learned policy, batch
    context); then for each of the n_classes four-step classes with the most
    points (transform length and prime range), every plan family of the
    class (each candidate shape of its longest product, each product taking
    that shape's fewest kept blocks) is put in the plan cache for the class's
    products, the other classes keeping the model's plans, and the whole
    batch is timed (median of three groups of k back-to-back launches)."""
    import collections

    import torch

    items = inputs.batch_uneven()
    lcs = [it.a.size + it.b.size - 1 for it in items]
    dev = torch.device("cuda")
    probs = [(torch.from_numpy(it.a).to(dev), torch.from_numpy(it.b).to(dev), it.p) for it in items]
    outs = [torch.empty(lc, dtype=torch.uint32, device=dev) for lc in lcs]
    pm.model_load(model)
    pm.set_policy(pm.POLICY_LEARNED)
    pm.plan_cache_clear()
    pb = pm.PreparedBatch(probs, outs=outs)
    pb.run()
    torch.cuda.synchronize()
    plans = pm.batch_plans_used(len(items))

    def timed():
        pb.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(k):
                pb.run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / k)
        return float(np.median(ts))

    base = timed()
    log(f"model's batch plans: {base:.4f} ms")
    cls = collections.defaultdict(list)
    for i, (it, P0) in enumerate(zip(items, plans)):
        if P0.kind == 2:
            cls[(P0.log_l, it.p != P)].append(i)
    top = sorted(cls, key=lambda key: -(len(cls[key]) << key[0]))[:n_classes]
    res = {"model_ms": base, "classes": []}
    for key in top:
        idx = cls[key]
        P0 = plans[idx[0]]
        fam0 = (P0.log_ra, P0.log_rb, P0.log_c, P0.lq, P0.lnt)
        i_max = max(idx, key=lambda i: lcs[i])
        fams = []
        for c in pm.plan_candidates(lcs[i_max], items[i_max].p, general_radix=False):
            f = (c.log_ra, c.log_rb, c.log_c, c.lq, c.lnt)
            if c.kind == 2 and f not in fams:
                fams.append(f)
        rows = []
        for f in fams:
            pm.plan_cache_clear()
            ok = True
            for i in idx:
                best = None
                for c in pm.plan_candidates(lcs[i], items[i].p, general_radix=False):
                    if c.kind == 2 and (c.log_ra, c.log_rb, c.log_c, c.lq, c.lnt) == f and (best is None or
                                                                                             c.ma < best.ma):
                        best = c
                if best is None:
                    ok = False
                    break
                pm.plan_cache_put(lcs[i], items[i].p, best)
            if ok:
                rows.append({"family": list(f), "ms": timed(), "model": f == fam0})
        pm.plan_cache_clear()
        best = min(rows, key=lambda r: r["ms"])
        entry = {"log_l": key[0], "prime_below_2^30": key[1], "products": len(idx), "model_family": list(fam0),
                 "best_family": best["family"], "best_ms": best["ms"], "families": rows}
        res["classes"].append(entry)
        log(f"class L = 2^{key[0]} ({'p < 2^30' if key[1] else 'p = 2013265921'}, {len(idx)} products): model "
            f"{fam0}, best {tuple(best['family'])} at {best['ms']:.4f} ms, {len(rows)} families")
    pm.set_policy(pm.POLICY_DEFAULT)
    if pm.stream_check() != 0:
        raise SystemExit("device error in the batch")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "batch_families.json"), "w") as f:
        json.dump(res, f, indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--quick", action="store_true", help="30 + 20 random lengths instead of 300 + 200")
    ap.add_argument("--model", help="evaluate this cost model (no tuning of the training lengths, no training)")
    ap.add_argument("--budget", type=float, help="seconds for the held-out loop; resume by running again")
    ap.add_argument("--batch-families", action="store_true",
                    help="only the whole-batch check of the model's batch plans (--model, default: the shipped "
                         "cost model): every plan family of the three largest classes timed on the whole batch")
    a = ap.parse_args(argv)
    if a.batch_families:
        import paper_1609_01010_amd as pm

        model = a.model or os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "cost_model.txt")
        batch_families(pm, model, a.out)
        return 0
    if run(a.out, reps=a.reps, steps=a.steps, quick=a.quick, model=a.model, budget=a.budget) is None:
        return 3
    return 0


if __name__ == "__main__":
    sys.exit(main())
