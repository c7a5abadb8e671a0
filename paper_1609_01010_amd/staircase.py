"""The power-of-two staircase, the truncated transform that smooths it, and
the general-radix lengths q 2^j, on one GPU (section 5, the comparison of
Fig. 3; section 1 for transforms of lengths other than powers of two).

For output lengths lc in {2^k - 1, 2^k + 1, 1.25 2^k, 1.5 2^k, 1.75 2^k},
k = kmin .. kmax, with p = 2013265921, every candidate plan is timed (the
tuner: median of `reps` runs each) and three libraries are compared, each
with its own fastest plan:

  * padded: both operands zero-padded to the next power of two L >= lc and
    the full length-L convolution (plans with n' = L): the paper's baseline;
  * relaxed TFT: any power-of-two plan, the truncated ones (n' = ma L / RA
    >= lc) included;
  * general radix: the products through a circular convolution of length
    q 2^j >= lc, q = 3, 5, 15 (the odd factors of p - 1), where it is
    shorter than L (plan kind 3).

The winners are then re-timed interleaved (three rounds of `reps` runs,
median of the medians), which removes the low bias of a minimum over many
noisy candidates.

Reported per length: the times, t(padded) / t(TFT) and which plan family the
tuner's whole space picks; overall, the geometric mean of t(padded) / t(TFT)
over the lengths that are not powers of two, and the lengths where a
general-radix plan beats the relaxed TFT.

    python -m paper_1609_01010_amd.staircase --out DIR [--reps 5] [--kmin 10] [--kmax 22]
"""

from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np

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


def nprime(plan, lc: int) -> int:
    if plan.kind == 0:
        return lc
    if plan.kind == 3:
        return plan.q << plan.log_l
    return plan.ma << (plan.log_l - plan.log_ra)


def run(out_dir: str, reps: int = 5, kmin: int = 10, kmax: int = 22):
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
        pow2 = [c for c in cands if c[1].kind != 3]
        padded = min((c for c in pow2 if nprime(c[1], lc) == L), key=lambda c: c[0])
        best = min(pow2, key=lambda c: c[0])
        gen = [c for c in cands if c[1].kind == 3]
        mixed = min(gen, key=lambda c: c[0]) if gen else None
        # interleaved re-timing of the winners
        tp, tt, tm = [], [], []
        for _ in range(3):
            tp.append(pm.time_plan(lc, P, padded[1], reps))
            tt.append(pm.time_plan(lc, P, best[1], reps))
            if mixed:
                tm.append(pm.time_plan(lc, P, mixed[1], reps))
        t_pad, t_tft = float(np.median(tp)), float(np.median(tt))
        t_mix = float(np.median(tm)) if mixed else None
        row = {"k": k, "lc": lc, "L": L, "padded_us": t_pad, "tft_us": t_tft,
               "padded_plan": list(padded[1].as_tuple()), "tft_plan": list(best[1].as_tuple()),
               "tft_nprime": nprime(best[1], lc), "ratio": t_pad / t_tft,
               "general_us": t_mix, "general_q": mixed[1].q if mixed else None,
               "general_n": nprime(mixed[1], lc) if mixed else None,
               "general_all_us": {f"{c[1].q}*2^{c[1].log_l}": c[0] for c in gen},
               "tuner_pick": "general" if (mixed and min(cands, key=lambda c: c[0])[1].kind == 3) else "pow2",
               "candidates": len(cands)}
        rows.append(row)
        mx = f"q={row['general_q']}: {t_mix:.1f} us" if mixed else "-"
        log(f"lc={lc} L={L} padded {t_pad:.1f} us  tft {t_tft:.1f} us  ratio {t_pad / t_tft:.2f}  general {mx}")
    pm.tune_db_clear()
    pm.plan_cache_clear()
    nonpow2 = [r for r in rows if r["lc"] & (r["lc"] - 1)]
    wins = [r for r in rows if r["general_us"] is not None and r["general_us"] < r["tft_us"]]
    summary = {
        "prime": P,
        "reps": reps,
        "lengths": len(rows),
        "geomean_padded_over_tft_nonpow2": float(np.exp(np.mean([math.log(r["ratio"]) for r in nonpow2]))),
        "by_shape": {},
        "general_radix_lengths": sum(r["general_us"] is not None for r in rows),
        "general_radix_beats_tft": [{"lc": r["lc"], "q": r["general_q"], "n": r["general_n"],
                                     "tft_over_general": r["tft_us"] / r["general_us"]} for r in wins],
    }
    for name, sel in (("2^k-1", lambda r: r["lc"] == (1 << r["k"]) - 1), ("2^k+1", lambda r: r["lc"] == (1 << r["k"]) + 1),
                      ("1.25*2^k", lambda r: r["lc"] == (1 << r["k"]) + (1 << r["k"]) // 4),
                      ("1.5*2^k", lambda r: r["lc"] == (1 << r["k"]) + (1 << r["k"]) // 2),
                      ("1.75*2^k", lambda r: r["lc"] == (1 << r["k"]) + 3 * (1 << r["k"]) // 4)):
        rs = [r for r in rows if sel(r)]
        summary["by_shape"][name] = float(np.exp(np.mean([math.log(r["ratio"]) for r in rs])))
    with open(os.path.join(out_dir, "staircase.json"), "w") as f:
        json.dump({"summary": summary, "rows": rows}, f, indent=1)
    lines = ["| lc | L | padded us | relaxed TFT us | padded / TFT | n' of the TFT plan | best q 2^j: n (us) | TFT / q 2^j |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        if r["general_us"] is not None:
            mx = f"{r['general_q']}: {r['general_n']} ({r['general_us']:.1f})"
            rg = f"{r['tft_us'] / r['general_us']:.2f}"
        else:
            mx, rg = "-", "-"
        lines.append(f"| {r['lc']} | 2^{int(math.log2(r['L']))} | {r['padded_us']:.1f} | {r['tft_us']:.1f} | "
                     f"{r['ratio']:.2f} | {r['tft_nprime']} | {mx} | {rg} |")
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
