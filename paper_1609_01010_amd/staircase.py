"""The power-of-two staircase and the truncated transform that smooths it, on
one GPU (section 5, the comparison of Fig. 3).

For output lengths lc in {2^k - 1, 2^k + 1, 1.25 2^k, 1.5 2^k, 1.75 2^k},
k = kmin .. kmax, with p = 2013265921, every candidate plan is timed (the
tuner: median of `reps` runs each) and two libraries are compared, each with
its own fastest plan:

  * padded: both operands zero-padded to the next power of two L >= lc and
    the full length-L convolution (plans with n' = L): the paper's baseline;
  * relaxed TFT: any plan, the truncated ones (n' = ma L / RA >= lc)
    included.

The two winners are then re-timed interleaved (three rounds of `reps` runs,
median of the medians), which removes the low bias of a minimum over many
noisy candidates.  Where a general-radix length q 2^j (q = 3, 5) lies
between lc and L, the product through it (pm_poly_mul_mixed) is timed too.

Reported per length: the three times and t(padded) / t(TFT); overall, the
geometric mean of that ratio over the lengths that are not powers of two.

    python -m paper_1609_01010_amd.staircase --out DIR [--reps 5] [--kmin 10] [--kmax 22]
"""

from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np

from . import inputs

P = 2013265921


def log(*a):
    print(*a, flush=True)


def lengths(kmin: int, kmax: int):
    out = []
    for k in range(kmin, kmax + 1):
        b = 1 << k
        for lc in (b - 1, b + 1, b + b // 4, b + b // 2, b + 3 * b // 4):
            out.append((k, lc))
    return out


def nprime(plan) -> int:
    return plan.ma << (plan.log_l - plan.log_ra)


def time_mixed(pm, torch, lc: int, q: int, reps: int) -> float:
    la, lb = inputs.split_output_length(lc)
    a, b = inputs.poly_pair((180, lc, q), la, lb, P)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    out = torch.empty(lc, dtype=torch.uint32, device="cuda")
    pm.poly_mul_mixed(ta, tb, P, q, out=out)
    ts = []
    for _ in range(3 * reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        pm.poly_mul_mixed(ta, tb, P, q, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return float(np.median(ts))


def run(out_dir: str, reps: int = 5, kmin: int = 10, kmax: int = 22):
    import torch

    import paper_1609_01010_amd as pm

    os.makedirs(out_dir, exist_ok=True)
    pm.lib()
    pm.set_policy(pm.POLICY_DEFAULT)
    rows = []
    for k, lc in lengths(kmin, kmax):
        L = 1 << math.ceil(math.log2(lc))
        pm.tune_db_clear()
        pm.plan_cache_clear()
        pm.tune([lc], P, reps=reps)
        cands = [(us, plan) for (l, p, plan, us) in pm.tune_db_rows() if l == lc and p == P]
        padded = min((c for c in cands if c[1].kind == 0 or nprime(c[1]) == L), key=lambda c: c[0])
        best = min(cands, key=lambda c: c[0])
        # interleaved re-timing of the two winners
        tp, tt = [], []
        for _ in range(3):
            tp.append(pm.time_plan(lc, P, padded[1], reps))
            tt.append(pm.time_plan(lc, P, best[1], reps))
        t_pad, t_tft = float(np.median(tp)), float(np.median(tt))
        mixed = {}
        for q in (3, 5):
            m = 1
            while q * m < lc:
                m *= 2
            if q * m < L and lc > 64:
                mixed[q] = time_mixed(pm, torch, lc, q, reps)
        row = {"k": k, "lc": lc, "L": L, "padded_us": t_pad, "tft_us": t_tft,
               "padded_plan": list(padded[1].as_tuple()), "tft_plan": list(best[1].as_tuple()),
               "tft_nprime": nprime(best[1]) if best[1].kind else lc,
               "ratio": t_pad / t_tft, "mixed_us": mixed, "candidates": len(cands)}
        rows.append(row)
        log(f"lc={lc} L={L} padded {t_pad:.1f} us  tft {t_tft:.1f} us  ratio {t_pad / t_tft:.2f}  "
            f"mixed {({q: round(v, 1) for q, v in mixed.items()})}")
    pm.tune_db_clear()
    pm.plan_cache_clear()
    nonpow2 = [r for r in rows if r["lc"] & (r["lc"] - 1)]
    summary = {
        "prime": P,
        "reps": reps,
        "lengths": len(rows),
        "geomean_padded_over_tft_nonpow2": float(np.exp(np.mean([math.log(r["ratio"]) for r in nonpow2]))),
        "by_shape": {},
    }
    for name, sel in (("2^k-1", lambda r: r["lc"] == (1 << r["k"]) - 1), ("2^k+1", lambda r: r["lc"] == (1 << r["k"]) + 1),
                      ("1.25*2^k", lambda r: r["lc"] == (1 << r["k"]) + (1 << r["k"]) // 4),
                      ("1.5*2^k", lambda r: r["lc"] == (1 << r["k"]) + (1 << r["k"]) // 2),
                      ("1.75*2^k", lambda r: r["lc"] == (1 << r["k"]) + 3 * (1 << r["k"]) // 4)):
        rs = [r for r in rows if sel(r)]
        summary["by_shape"][name] = float(np.exp(np.mean([math.log(r["ratio"]) for r in rs])))
    with open(os.path.join(out_dir, "staircase.json"), "w") as f:
        json.dump({"summary": summary, "rows": rows}, f, indent=1)
    lines = ["| lc | L | padded us | relaxed TFT us | padded / TFT | n' of the TFT plan | q 2^j (us) |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        mx = ", ".join(f"q={q}: {v:.1f}" for q, v in r["mixed_us"].items()) or "-"
        lines.append(f"| {r['lc']} | 2^{int(math.log2(r['L']))} | {r['padded_us']:.1f} | {r['tft_us']:.1f} | "
                     f"{r['ratio']:.2f} | {r['tft_nprime']} | {mx} |")
    with open(os.path.join(out_dir, "staircase.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    log(json.dumps(summary))
    return summary


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--kmin", type=int, default=10)
    ap.add_argument("--kmax", type=int, default=22)
    a = ap.parse_args()
    run(a.out, a.reps, a.kmin, a.kmax)


if __name__ == "__main__":
    main()
