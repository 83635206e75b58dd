#!/usr/bin/env python
"""Throughput benchmark of the MI355X DECO library on one GPU.

Workload: full pDECO (unlifted/lifted alternation, importance-based degree start,
evolutionary search over the two step sizes and the lift dimension with a population of
8) on a Barabasi-Albert graph n = 10,000, m = 4, unit weights, B = 256 initialisations.
A "step" of this benchmark is one lift-and-project round: T_q unlifted gradient steps and
T_l lifted gradient steps (each fused with rounding, exact scoring of every iterate and the
running best), the lift, the projection and one evolution update.

Reported value: edge-updates/s = sum over gradient steps of nnz * columns, divided by the
wall time of the timed rounds (inputs resident in HBM). Also reported: the live roofline of
the step kernels (HIP events on the library's stream), the CPU oracle timed on this host's
cores on a bounded sample, and time-to-cut (0.995 of the plain float32 method's best) for
float32 and bfloat16 storage of X.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-updates/s (nnz·B·steps/s); time-to-cut within 0.5% of best, plain vs chosen"
HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_ba10k_B256_bf16_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2509_18612_amd", "csrc", "kernels.hip")


def measured_traffic(which):
    """Fabric bytes per launch of a step-kernel shape from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the factor a copy of known size gives), or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ":" in ln and ln.startswith("- "):
            k, v = ln[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernels.hip sha256") != sha:
        return None
    v = vals.get(f"traffic bytes per launch ({which})")
    return int(v) if v else None


def algorithmic_bytes(n, nnz, C, G, s_x, s_w):
    """Minimum HBM bytes of one fused step: row_ptr, col_idx (+ weights), X_t read once,
    X_t+1 written once, one double per (graph, column) of cut results."""
    return 4 * (n + G) + (4 + s_w) * nnz + 2 * s_x * n * C + 8 * C * G


def time_step_kernel(deco, torch, G, B, l, dtype, steps, eta=0.01, seed=1):
    """Average duration per launch of the fused step kernel, HIP events on its stream."""
    lifted = l > 1
    h = deco.Handle(G, B=B, l=l, lifted=lifted, x_dtype=dtype, eta=eta, seed=seed)
    h.start(deco.INIT_IDI, scale=1e4, sigma2=0.8, batch=0)
    h.step(steps, use_graph=True)  # capture + warm
    h.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    h.step(steps, use_graph=True)
    e1.record(h.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sched = h.schedule()
    h.destroy()
    return ms, sched


def time_handle(torch, h, steps, kind, **start):
    """Average per-launch time (us) of h's step kernel, HIP events on its stream."""
    h.start(kind, **start)
    h.step(steps, use_graph=True)
    h.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    h.step(steps, use_graph=True)
    e1.record(h.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps * 1e3


def other_workloads(deco, synth, torch, which):
    """Step-kernel measurements on the other workload shapes (not the benchmark value)."""
    import numpy as np
    out = {}
    if "er800" in which:
        g = synth.erdos_renyi(800, 0.06, 0)
        h = deco.Handle(deco.Graph(g), B=16, eta=0.1)
        us = time_handle(torch, h, 200, deco.INIT_UNIFORM)
        A = algorithmic_bytes(g.n, g.nnz, 16, 1, 4, 0)
        out["er800_B16_f32"] = {"us_per_step": round(us, 3), "edge_updates_per_s": g.nnz * 16 / us * 1e6,
                                "hbm_frac": round(A / us / 1e3 / HBM_PEAK_GBS, 4), "schedule": h.schedule()}
        h.destroy()
    if "uneven" in which:
        g = synth.uneven_batch(512, 7)
        h = deco.Handle(deco.Graph(g), B=64, x_dtype=deco.BF16, eta=0.01)
        h.autotune(5)
        us = time_handle(torch, h, 50, deco.INIT_IDI, scale=1e4, sigma2=0.8)
        A = algorithmic_bytes(g.n, g.nnz, 64, 512, 2, 0)
        out["uneven512_B64_bf16"] = {"us_per_step": round(us, 2), "edge_updates_per_s": g.nnz * 64 / us * 1e6,
                                     "hbm_frac": round(A / us / 1e3 / HBM_PEAK_GBS, 4), "n": g.n, "nnz": g.nnz,
                                     "schedule": h.schedule()}
        h.destroy()
    if "reg3" in which:
        g = synth.with_rademacher_weights(synth.random_regular3(1_000_000, 0), 3)
        h = deco.Handle(deco.Graph(g), B=128, x_dtype=deco.BF16, eta=0.01)
        h.autotune(5)
        us = time_handle(torch, h, 40, deco.INIT_UNIFORM)
        A = algorithmic_bytes(g.n, g.nnz, 128, 1, 2, 4)
        out["reg3_1e6_pm1_B128_bf16"] = {"us_per_step": round(us, 2), "edge_updates_per_s": g.nnz * 128 / us * 1e6,
                                         "achieved_GBs": round(A / us / 1e3, 1),
                                         "hbm_frac": round(A / us / 1e3 / HBM_PEAK_GBS, 4),
                                         "bytes_per_launch": A, "schedule": h.schedule()}
        h.destroy()
    if "dense" in which:
        g = synth.erdos_renyi(8192, 0.5, 0)
        W = torch.zeros((g.n, g.n), dtype=torch.float32, device="cuda")
        rows = torch.from_numpy(np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))).cuda()
        W[rows, torch.from_numpy(g.col_idx.astype(np.int64)).cuda()] = 1.0
        Wb = W.to(torch.bfloat16)
        del W
        h = deco.DenseHandle(Wb, B=512, eta=0.01)
        us = time_handle(torch, h, 20, deco.INIT_UNIFORM)
        flop = 2.0 * 2 * g.n * g.n * 512  # W X and W sign(X)
        tf = flop / us / 1e6
        out["dense_er8192_B512_bf16_mfma"] = {"us_per_step": round(us, 2), "tflops": round(tf, 1),
                                              "mfma_frac_bf16_dense": round(tf / 2500.0, 4),
                                              "edge_updates_per_s": g.nnz * 512 / us * 1e6,
                                              "flop_per_launch": flop}
        h.destroy()
    return out


def kernel_only(deco, torch, G, B, l_max, dtype, args):
    """Counter runs: the step kernel of one bench shape with its autotuned schedule, or a
    plain 256 MiB device-to-device copy (the calibration of the traffic counters)."""
    if args.kernel_only == "copy":
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.kernel_steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# copied {a.numel() * 4} bytes x {args.kernel_steps}", flush=True)
        return
    l = 1 if args.kernel_only == "unlifted" else l_max
    h = deco.Handle(G, B=B, l=l, lifted=l > 1, x_dtype=dtype, eta=0.01, seed=1)
    h.autotune(10)
    h.start(deco.INIT_IDI, scale=1e4, sigma2=0.8, batch=0)
    h.synchronize()
    h.step(args.kernel_steps)
    h.synchronize()
    print(f"# {args.kernel_only}: {args.kernel_steps} launches, schedule {h.schedule()}", flush=True)
    h.destroy()


def cpu_baseline(oracle, csr, B, budget_s):
    """The oracle's batch (step + rounding + exact cut + running best per step, FP64,
    one thread) on the same graph, for as many steps as fit in about budget_s seconds."""
    import numpy as np
    g = oracle.Graph(csr)
    x0 = np.random.default_rng(0).uniform(-1e-4, 1e-4, (csr.n, B))
    t0 = time.perf_counter()
    oracle.run_batch(g, x0, B, 1, False, 0.01, 1)
    one = time.perf_counter() - t0
    k = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    oracle.run_batch(g, x0, B, 1, False, 0.01, k)
    dt = time.perf_counter() - t0
    return csr.nnz * B * k / dt, k, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed lift-and-project rounds")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--storage", choices=["bf16", "f32"], default="bf16")
    ap.add_argument("--B", type=int, default=256)
    ap.add_argument("--Tq", type=int, default=1000)
    ap.add_argument("--Tl", type=int, default=400)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttc", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--others", default="er800,uneven,reg3,dense",
                    help="comma list of other workload shapes to time (empty: none)")
    ap.add_argument("--kernel-only", choices=["unlifted", "lifted", "copy"], default=None,
                    help="run only the step kernel of that shape (autotuned as in the bench) for "
                         "--kernel-steps launches, or a 256 MiB device copy, for counter runs")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_18612_amd import deco, synth

    torch.cuda.set_device(0)
    n, m, B = 10_000, 4, args.B
    csr = synth.barabasi_albert(n, m, 0)
    G = deco.Graph(csr)
    dtype = deco.BF16 if args.storage == "bf16" else deco.F32
    K, l_max = 8, 4
    if args.kernel_only:
        kernel_only(deco, torch, G, B, l_max, dtype, args)
        return
    print(f"# graph BA({n},{m}) nnz={csr.nnz}; B={B}; storage={args.storage}", file=sys.stderr, flush=True)

    # the first solver of a shape autotunes both step kernels; later handles of the same
    # shape (the kernel timing and time-to-cut below) reuse the cached winner
    solver = deco.Solver(G, B=B, K=K, l_max=l_max, evo_rounds=2, T_q=args.Tq, T_l=args.Tl, x_dtype=dtype,
                         init_kind=deco.INIT_IDI, seed=0, use_graph=True, autotune=not args.no_autotune)
    w = solver.run(args.warmup) if args.warmup > 0 else None
    eu0 = w["edge_updates"] if w else 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = solver.run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solver.destroy()
    dt = t1 - t0
    eu = res["edge_updates"] - eu0
    value = eu / dt
    print(f"# timed {args.steps} rounds in {dt:.3f}s; best cut {res['best_cut'][0]:.0f}", file=sys.stderr,
          flush=True)

    # live roofline of the two step-kernel shapes of a round
    s_x = 2 if dtype == deco.BF16 else 4
    ms_q, sched_q = time_step_kernel(deco, torch, G, B, 1, dtype, args.kernel_steps)
    ms_l, sched_l = time_step_kernel(deco, torch, G, B, l_max, dtype, args.kernel_steps)
    A_q = algorithmic_bytes(n, csr.nnz, B, 1, s_x, 0)
    A_l = algorithmic_bytes(n, csr.nnz, B * l_max, 1, s_x, 0)
    share_q = args.Tq * ms_q
    share_l = args.Tl * ms_l
    dom_ms, dom_A, dom_name = (ms_l, A_l, f"k_step lifted l={l_max}") if share_l >= share_q else \
        (ms_q, A_q, "k_step unlifted")
    achieved = dom_A / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("lifted" if dom_name.startswith("k_step lifted") else "unlifted"),
                "kernel": dom_name, "bytes_per_launch": dom_A, "us_per_launch": round(dom_ms * 1e3, 3)}

    cpu = None
    if not args.no_cpu:
        import oracle
        v, k, cdt = cpu_baseline(oracle, csr, B, args.cpu_seconds)
        cpu = {"value": v, "unit": "edge-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} oracle steps (FP64 step + rounding + exact cut + running best, unlifted, "
                         f"B={B}) on the same BA graph, {cdt:.1f}s on 1 thread"}

    others = other_workloads(deco, synth, torch, set(filter(None, args.others.split(","))))
    ttc = None
    if not args.no_ttc:
        ttc = time_to_cut(deco, torch, G, B, K, l_max, args)

    line = {
        "metric": METRIC, "value": value, "unit": "edge-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / max(res["rounds_done"], 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"pDECO on BA(n={n},m={m}) unit weights, B={B}, population {K}, l_max={l_max}, "
                               f"T_q={args.Tq}, T_l={args.Tl} per round",
                   "x_storage": args.storage, "accumulate": "f32", "global_batch": B, "graphs": 1,
                   "nnz": csr.nnz},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_cut": ttc,
        "extra": {"step_kernel_us": {"unlifted": round(ms_q * 1e3, 3), "lifted": round(ms_l * 1e3, 3)},
                  "hbm_frac": {"unlifted": round(A_q / (ms_q * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "lifted": round(A_l / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                  "schedule": {"unlifted": sched_q, "lifted": sched_l},
                  "best_cut": float(res["best_cut"][0]), "genes": [res["eq_best"], res["el_best"], res["l_best"]],
                  "workloads": others},
    }
    print(json.dumps(line), flush=True)


def time_to_cut(deco, torch, G, B, K, l_max, args):
    """Reference: plain float32 pDECO for a fixed 8 rounds gives best_plain; target = 0.995
    best_plain. Each variant is timed from solver creation to the first round whose best
    reaches the target (at most 12 rounds)."""
    import numpy as np
    ref = deco.Solver(G, B=B, K=K, l_max=l_max, evo_rounds=2, T_q=args.Tq, T_l=args.Tl, x_dtype=deco.F32,
                      init_kind=deco.INIT_IDI, seed=1, use_graph=True, autotune=not args.no_autotune)
    r = ref.run(8)
    ref.destroy()
    best_plain = float(r["best_cut"][0])
    target = 0.995 * best_plain
    out = {"best_plain_f32": best_plain, "target": target, "reference_rounds": 8}
    for name, dt in [("f32", deco.F32), ("bf16", deco.BF16)]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = deco.Solver(G, B=B, K=K, l_max=l_max, evo_rounds=2, T_q=args.Tq, T_l=args.Tl, x_dtype=dt,
                        init_kind=deco.INIT_IDI, seed=2, use_graph=True, target_cut=[target],
                        autotune=not args.no_autotune)
        rr = s.run(12)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.destroy()
        reached = bool(rr["best_cut"][0] >= target)
        out[name] = {"seconds": t1 - t0 if reached else None, "reached": reached,
                     "rounds": rr["rounds_done"], "best": float(rr["best_cut"][0])}
    return out


if __name__ == "__main__":
    main()
