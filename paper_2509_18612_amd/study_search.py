"""Manual against automatic selection of the step size and step count (the study of the
paper's appendix on the parameter search: Table FX gives the manual (alpha, T) tuples, the
automatic runs use the evolutionary search of Sec. 4.3 with population 6 and 5 evolution
rounds, T in [3000, 10000] and log10 alpha in [-4, -1]).

Synthetic stand-ins for the paper's small ER set (n in 700..800, p = 0.15): ER graphs drawn
by the package's generator; the paper's own instances are not available, so the cut values
are comparable in shape only. Each graph runs pQUCO (unlifted batches only), pLUCO (lifted
batches only, l = 2) and pDECO (lift-and-project rounds) with the manual tuples and with the
search, B initialisations, importance-based start (beta 0.2), exploration variance 0.8 and
1e-4 scaling (Sec. 5); reported: mean best cut and mean wall time per graph.

    python -m paper_2509_18612_amd.study_search --graphs 16 --out R.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import deco, synth

# Table FX, small ER row: (alpha, T) per method; pDECO has one tuple per formulation
MANUAL = {"pQUCO": ((0.15, 48000),), "pLUCO": ((0.001, 2500),), "pDECO": ((0.10, 30000), (0.001, 2000))}
MODE = {"pQUCO": deco.SOLVE_UNLIFTED, "pLUCO": deco.SOLVE_LIFTED, "pDECO": deco.SOLVE_DECO}


def run(G, method, automatic, B, seed, x_dtype):
    import torch
    kw = dict(B=B, l_max=2, x_dtype=x_dtype, seed=seed, use_graph=True, mode=MODE[method], init_kind=deco.INIT_IDI,
              beta=0.2, sigma2=0.8, scale=1e4)
    if automatic:
        K, evo = 6, 5
        kw.update(K=K, rounds=evo + 1, evo_rounds=evo, T_q=10000, T_l=10000, T_min=3000, T_l_min=3000,
                  l0=[2] * K)
    else:
        tup = MANUAL[method]
        q = tup[0] if method != "pLUCO" else None
        l_ = tup[-1] if method != "pQUCO" else None
        kw.update(K=1, rounds=1, evo_rounds=0, T_q=q[1] if q else 1, T_l=l_[1] if l_ else 1,
                  eq0=[math.log10(q[0]) if q else -2.0], el0=[math.log10(l_[0]) if l_ else -3.0], l0=[2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = deco.solve(G, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    genes = {"eq": r["eq_best"], "el": r["el_best"], "l": r["l_best"], "T_q": r["T_best"], "T_l": r["T_l_best"]}
    return float(r["best_cut"][0]), dt, int(r["steps_done"]), genes


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--graphs", type=int, default=16)
    ap.add_argument("--B", type=int, default=48, help="initialisations per graph (a multiple of 6 and of 8)")
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    x_dtype = deco.F32 if args.dtype == "f32" else deco.BF16
    rng = np.random.default_rng(args.seed)
    sizes = [int(rng.integers(700, 801)) for _ in range(args.graphs)]
    rows = []
    t_start = time.time()
    for i, n in enumerate(sizes):
        g = synth.erdos_renyi(n, 0.15, 4_000_000 + i)
        G = deco.Graph(g)
        run(G, "pQUCO", False, args.B, 0, x_dtype)  # warm the kernels and the schedule cache of this shape
        for method in ("pQUCO", "pLUCO", "pDECO"):
            for automatic in (False, True):
                cut, dt, steps, genes = run(G, method, automatic, args.B, 100 + i, x_dtype)
                rows.append({"graph": i, "n": n, "nnz": g.nnz, "method": method,
                             "selection": "automatic" if automatic else "manual", "cut": cut, "seconds": dt,
                             "steps": steps, "genes": genes})
        print(f"[{time.time() - t_start:6.1f}s] graph {i} (n={n}): " +
              ", ".join(f"{r['method']}/{r['selection'][0]} {r['cut']:.0f}" for r in rows[-6:]), flush=True)
    table = {}
    for method in ("pQUCO", "pLUCO", "pDECO"):
        for sel in ("manual", "automatic"):
            rs = [r for r in rows if r["method"] == method and r["selection"] == sel]
            table[f"{method} {sel}"] = {"mean_cut": float(np.mean([r["cut"] for r in rs])),
                                        "mean_seconds": float(np.mean([r["seconds"] for r in rs])),
                                        "mean_steps": float(np.mean([r["steps"] for r in rs]))}
    out = {"protocol": {"graphs": args.graphs, "family": "ER(n~U{700..800}, 0.15)", "B": args.B,
                        "dtype": args.dtype, "manual": MANUAL,
                        "automatic": "population 6, 5 evolution rounds then 1 round with the best genes, "
                                     "T in [3000, 10000], log10 alpha in [-4, -1], l starts at 2 (l_max 2)"},
           "table": table, "rows": rows}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(table, indent=1), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
