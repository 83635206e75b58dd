"""Learned starting magnitudes (DECO_INIT_LEARNED): training data, GPU training and evaluation.

The paper's method is training-free; this is the learned-start extension. A 3-layer
message-passing network (deco_mpnn_*) maps per-node degree features to a magnitude y_v in
(0, 1); the start's mean is y_v times the importance-based sign of Sec. 4.1, then the usual
exploration noise and 1/s scaling of Sec. 4.2 and Sec. 5.

Protocol (run as a module; every step runs on the GPU through the library):
  training graphs  Barabasi-Albert, n ~ U{500..5000}, m ~ U{2..6}
  labels           t_v = fraction of v's edge weight cut by the best vector that plain pDECO
                   (importance-based start, the library's solver) finds for the graph
  training         mean squared error, Adam, on block-diagonal batches of training graphs
  evaluation       held-out BA(n = 20,000, m ~ U{2..6}) and ER(5000, 0.002) graphs, B = 128:
                   steps of the unlifted batch (Alg. 1, the stage the start feeds) until the
                   graph's running best reaches a target, for the importance-based start and the
                   learned start with the same seed (paired); targets 0.995 of the graph's best
                   plain pDECO cut and 0.995 of the best of a long unlifted batch from the
                   importance-based start (another seed). Reported with paired 95% intervals.

    python -m paper_2509_18612_amd.learned --out-weights W.npy --out-report R.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import deco, synth

HID, IN = 64, 3


SHAPES = [("ws1", (IN, HID)), ("wn1", (IN, HID)), ("b1", (HID,)), ("ws2", (HID, HID)), ("wn2", (HID, HID)),
          ("b2", (HID,)), ("ws3", (HID, HID)), ("wn3", (HID, HID)), ("b3", (HID,)), ("wo", (HID,)), ("bo", (1,))]


def glorot_params(seed: int) -> np.ndarray:
    """Packed parameters in the library's order: Glorot-uniform matrices (the head's weights
    as a 64 x 1 matrix), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shp in SHAPES:
        if name.startswith("b"):
            out.append(np.zeros(shp, np.float32))
        else:
            fan_out = shp[1] if len(shp) > 1 else 1
            lim = np.sqrt(6.0 / (shp[0] + fan_out))
            out.append(rng.uniform(-lim, lim, shp).astype(np.float32))
    return np.concatenate([o.reshape(-1) for o in out])


def _ba(args):
    n, m, seed = args
    return synth.barabasi_albert(n, m, seed)


def _er(args):
    n, p, seed = args
    return synth.erdos_renyi(n, p, seed)


def _workers():
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, usable))


def make_graphs(fn, specs):
    with ProcessPoolExecutor(_workers()) as ex:
        return list(ex.map(fn, specs, chunksize=4))


def training_specs(count, seed):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(500, 5001)), int(rng.integers(2, 7)), 1_000_000 + seed * 10_000 + i)
            for i in range(count)]


def chunks(items, size):
    return [items[i:i + size] for i in range(0, len(items), size)]


def label_batches(graphs, per_batch, seed, B=64, rounds=3, T_q=300, T_l=100):
    """Block-diagonal batches with the labels of plain pDECO's best vector per graph."""
    out = []
    for i, part in enumerate(chunks(graphs, per_batch)):
        G = deco.Graph(synth.block_diagonal(part))
        r = deco.solve(G, B=B, K=8, l_max=2, rounds=rounds, evo_rounds=2, T_q=T_q, T_l=T_l, seed=seed + i,
                       x_dtype=deco.BF16)
        out.append((G, deco.Mpnn().labels(G, r["z"])))
    return out


def train(net, batches, epochs, lr, log=print):
    losses = []
    for ep in range(epochs):
        ls = []
        for G, t in batches:
            ls.append(net.loss_grad(G, t))
            net.adam(lr)
        losses.append(float(np.mean(ls)))
        log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses


def validation_loss(net, batches):
    import torch
    vals = []
    for G, t in batches:
        y = net.forward(G)
        vals.append(float(torch.mean((y - t) ** 2).item()))
    return float(np.mean(vals))


def unlifted_trace(G, B, T, kind, seed, eta, magnitude=None):
    """Running best cut per graph after each step of one unlifted batch ([T+1, G])."""
    h = deco.Handle(G, B=B, eta=eta, seed=seed)
    h.start(kind, scale=1e4, sigma2=0.8, batch=0, magnitude=magnitude)
    tr = h.set_trace(T + 1)
    h.step(T, use_graph=True)
    h.round_score()
    best = np.maximum.accumulate(tr.cpu().numpy().max(axis=2), axis=0)
    h.destroy()
    return best


def first_hit(best, target):
    """First step at which each graph's running best reaches its target (-1: never)."""
    hit = best >= target[None, :]
    first = np.argmax(hit, axis=0)
    return np.where(hit.any(axis=0), first, -1)


def paired_ci(d):
    d = np.asarray(d, np.float64)
    if d.size < 2:
        return None
    m = float(d.mean())
    h = float(1.96 * d.std(ddof=1) / np.sqrt(d.size))
    return {"mean": m, "lo": m - h, "hi": m + h, "n": int(d.size)}


def evaluate(net, graphs, per_batch, B, T, eta, seed, ref_rounds=3, log=print, normalise=False):
    """Per-graph steps to the targets for the importance-based and the learned start."""
    rows = []
    for i, part in enumerate(chunks(graphs, per_batch)):
        G = deco.Graph(synth.block_diagonal(part))
        ref = deco.solve(G, B=B, K=8, l_max=2, rounds=ref_rounds, evo_rounds=2, T_q=600, T_l=200, seed=seed + i,
                         x_dtype=deco.BF16)
        long_best = unlifted_trace(G, B, 2 * T, deco.INIT_IDI, seed + 7919 + i, eta)[-1]
        y = net.forward(G)
        b_idi = unlifted_trace(G, B, T, deco.INIT_IDI, seed + 104729 + i, eta)
        b_lrn = unlifted_trace(G, B, T, deco.INIT_LEARNED, seed + 104729 + i, eta, magnitude=y)
        if normalise:
            # magnitudes divided by their per-graph mean (the start keeps IDI's mean size)
            import torch
            off = np.asarray(G.csr.graph_row_offset, np.int64)
            counts = torch.from_numpy(np.diff(off)).to(y.device)
            gid = torch.repeat_interleave(torch.arange(len(part), device=y.device), counts)
            mean = torch.zeros(len(part), device=y.device).index_add_(0, gid, y) / counts.float()
            b_lrn = unlifted_trace(G, B, T, deco.INIT_LEARNED, seed + 104729 + i, eta, magnitude=y / mean[gid])
        for tname, tv in (("deco", 0.995 * ref["best_cut"]), ("batch", 0.995 * long_best)):
            s_i, s_l = first_hit(b_idi, tv), first_hit(b_lrn, tv)
            for gi in range(len(part)):
                rows.append({"batch": i, "graph": gi, "target_kind": tname, "target": float(tv[gi]),
                             "steps_idi": int(s_i[gi]), "steps_learned": int(s_l[gi]),
                             "final_idi": float(b_idi[-1, gi]), "final_learned": float(b_lrn[-1, gi]),
                             "step0_idi": float(b_idi[0, gi]), "step0_learned": float(b_lrn[0, gi])})
        log(f"eval batch {i}: {len(part)} graphs")
    return rows


def summarise(rows, T):
    out = {}
    for tname in ("deco", "batch"):
        rs = [r for r in rows if r["target_kind"] == tname]
        both = [r for r in rs if r["steps_idi"] >= 0 and r["steps_learned"] >= 0]
        # a run that never reaches the target counts as T + 1 steps in the censored comparison
        cens = [(r["steps_idi"] if r["steps_idi"] >= 0 else T + 1) - (r["steps_learned"] if r["steps_learned"] >= 0
                                                                      else T + 1) for r in rs]
        out[tname] = {
            "graphs": len(rs),
            "reached_idi": sum(r["steps_idi"] >= 0 for r in rs),
            "reached_learned": sum(r["steps_learned"] >= 0 for r in rs),
            "median_steps_idi": float(np.median([r["steps_idi"] for r in both])) if both else None,
            "median_steps_learned": float(np.median([r["steps_learned"] for r in both])) if both else None,
            "steps_saved_when_both_reach": paired_ci([r["steps_idi"] - r["steps_learned"] for r in both]),
            "steps_saved_censored": paired_ci(cens),
            "learned_fewer": sum(c > 0 for c in cens), "learned_more": sum(c < 0 for c in cens),
            "ties": sum(c == 0 for c in cens),
        }
    rs = [r for r in rows if r["target_kind"] == "deco"]
    out["final_best_learned_minus_idi"] = paired_ci([r["final_learned"] - r["final_idi"] for r in rs])
    out["start_cut_learned_minus_idi"] = paired_ci([r["step0_learned"] - r["step0_idi"] for r in rs])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-graphs", type=int, default=2000)
    ap.add_argument("--per-batch", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-ba", type=int, default=200)
    ap.add_argument("--eval-er", type=int, default=200)
    ap.add_argument("--eval-B", type=int, default=128)
    ap.add_argument("--eval-T", type=int, default=1000)
    ap.add_argument("--eval-eta", type=float, default=10 ** -1.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--load-weights", default="", help="evaluate these weights instead of training")
    ap.add_argument("--normalise", action="store_true", help="evaluate magnitudes divided by their graph mean")
    ap.add_argument("--out-weights", default="")
    ap.add_argument("--out-report", required=True)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    t_start = time.time()

    def log(msg):
        print(f"[{time.time() - t_start:7.1f}s] {msg}", flush=True)

    if args.load_weights:
        net = deco.Mpnn(np.load(args.load_weights, allow_pickle=False))
        graphs, trn, nval, losses, v0, v1, train_s = [], [], 0, [], None, None, 0.0
    else:
        specs = training_specs(args.train_graphs, args.seed)
        graphs = make_graphs(_ba, specs)
        log(f"{len(graphs)} training graphs, {sum(g.n for g in graphs)} nodes")
        batches = label_batches(graphs, args.per_batch, seed=args.seed * 1000 + 17)
        nval = max(1, len(batches) // 20)
        val, trn = batches[:nval], batches[nval:]
        log(f"labels: {len(batches)} batches ({nval} held out for validation)")
        net = deco.Mpnn(glorot_params(args.seed))
        v0 = validation_loss(net, val)
        t0 = time.time()
        losses = train(net, trn, args.epochs, args.lr, log=log)
        train_s = time.time() - t0
        v1 = validation_loss(net, val)
        log(f"validation loss {v0:.5f} -> {v1:.5f}; training {train_s:.1f}s")
        if args.out_weights:
            os.makedirs(os.path.dirname(os.path.abspath(args.out_weights)), exist_ok=True)
            np.save(args.out_weights, net.params.cpu().numpy().astype(np.float32))

    rng = np.random.default_rng(args.seed + 99)
    ba_specs = [(20_000, int(rng.integers(2, 7)), 2_000_000 + i) for i in range(args.eval_ba)]
    er_specs = [(5000, 0.002, 3_000_000 + i) for i in range(args.eval_er)]
    ba = make_graphs(_ba, ba_specs)
    er = make_graphs(_er, er_specs)
    log(f"evaluation graphs: {len(ba)} BA(20000), {len(er)} ER(5000, 0.002)")
    rows_ba = evaluate(net, ba, 20, args.eval_B, args.eval_T, args.eval_eta, 5000, log=log, normalise=args.normalise)
    rows_er = evaluate(net, er, 50, args.eval_B, args.eval_T, args.eval_eta, 6000, log=log, normalise=args.normalise)
    report = {
        "protocol": {"train_graphs": len(graphs), "train_family": "BA(n~U{500..5000}, m~U{2..6})",
                     "labels": "plain pDECO best vector per graph (B=64, K=8, l_max=2, 3 rounds, T_q=300, T_l=100)",
                     "epochs": args.epochs, "lr": args.lr, "batches": len(trn), "validation_batches": nval,
                     "normalised_magnitudes": bool(args.normalise),
                     "eval": {"ba": f"{len(ba)} x BA(20000, m~U{{2..6}})", "er": f"{len(er)} x ER(5000, 0.002)",
                              "B": args.eval_B, "T": args.eval_T, "eta": args.eval_eta,
                              "start": "scale 1e4, sigma2 0.8, same seed for both starts"}},
        "training": {"loss_per_epoch": losses, "validation_before": v0, "validation_after": v1,
                     "seconds": train_s},
        "ba": summarise(rows_ba, args.eval_T), "er": summarise(rows_er, args.eval_T),
        "seconds_total": time.time() - t_start,
    }
    with open(args.out_report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps({"ba": report["ba"], "er": report["er"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
