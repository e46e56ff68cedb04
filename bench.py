"""Throughput of the TreeRay/OnTheSpot hot path on one MI355X.

A step is one outer iteration over the whole grid: point-source deposit,
cell quantities, FP64 node moments, the sweep (walk + node->ray mapping +
per-ray On-the-Spot integration + sum over rays) and delta_cell.  Inputs
(densities, previous flux) are resident in HBM before the timed region.

The workload is the uniform 64^3 grid around one Q = 1e49 source with
N_side 4 (192 rays), theta 0.5 and 48 evaluation points.  The FP32 +
compensated form is timed for `value`; the FP64 form runs the same steps on
the same inputs for the speed-up.  The FP64 CPU oracle is timed on a bounded
sample of targets on the host and gives the reported error of both forms.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target-cell·ray updates/s, FP32-compensated vs FP64, at ≤1e-4 rel flux err"
HBM_PEAK_GBS = 8000.0
# node bytes of the sweep: walk test (int4 geometry + int2 topology), mapping
# (two 4-vectors of moments) in the precision of the form
WALK_BYTES = 24
MAP_BYTES = {"f32": 32, "f64": 64}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="workload: 1, 2 or 3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=98304, help="oracle targets in the CPU baseline")
    ap.add_argument("--no-autotune", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2105_09644_amd as T
    from paper_2105_09644_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    T.load_library()
    P = W.CONFIGS[args.config]()
    npix = 12 * P.params.nside ** 2
    n_cells = P.total_cells()
    nh = torch.tensor(np.concatenate(P.n_h), dtype=torch.float64, device="cuda")

    def run_form(prec):
        ctx = T.context_for(P, prec)
        f_prev = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
        f_new = torch.zeros_like(f_prev)
        ion = torch.zeros(n_cells, dtype=torch.uint8, device="cuda")
        ctx.build(nh, None, thin=True)
        ctx.sweep(f_prev, ion)
        ctx.build(nh, f_prev)
        if not args.no_autotune:
            ctx.autotune()
        for _ in range(args.warmup):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)
            ctx.delta(f_new, f_prev)
        torch.cuda.synchronize()
        sweep_ms = []
        acc = tested = 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)
            ctx.delta(f_new, f_prev)     # synchronises the stream
            st = ctx.stats()
            sweep_ms.append(st.last_sweep_ms)
            acc, tested = st.nodes_accepted, st.nodes_tested
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = ctx.stats()
        res = dict(ms_per_step=dt * 1e3, value=n_cells * npix / dt, sweep_ms=float(np.mean(sweep_ms)),
                   accepted=int(acc), tested=int(tested), waves=st.waves_per_target,
                   per_cu=st.targets_per_cu, guard=int(st.guard_recomputes))
        # parity input independent of either side: an absorbing sweep with zero previous flux
        ctx.build(nh, None)
        ctx.sweep(f_new, ion)
        ctx.sync()
        res["flux0"] = f_new.cpu().numpy()
        ctx.close()
        return res

    r32 = run_form(T.TR_FP32C)
    r64 = run_form(T.TR_FP64)

    # roofline of the sweep kernel: the interaction-list bytes (no reuse credited)
    def roof(r, form):
        byts = r["tested"] * WALK_BYTES + r["accepted"] * MAP_BYTES[form] + n_cells * 9
        gbs = byts / (r["sweep_ms"] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_sweep", "bytes_per_launch": int(byts), "launch_ms": round(r["sweep_ms"], 3)}

    line = {
        "metric": METRIC,
        "value": round(r32["value"], 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": P.name, "cells": n_cells, "n_pix": npix, "theta": P.params.theta,
                   "n_radial": P.params.n_radial, "precision": "FP32 walk/weights/ray buffers, FP64 moments "
                   "and ray integration, compensated sums"},
        "fp64": {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 3),
                 "sweep_ms": round(r64["sweep_ms"], 3)},
        "speedup_vs_fp64": round(r32["value"] / r64["value"], 3),
        "sweep_ms": round(r32["sweep_ms"], 3),
        "launch": {"fp32c_waves_per_target": r32["waves"], "fp32c_targets_per_cu": r32["per_cu"],
                   "fp64_waves_per_target": r64["waves"], "fp64_targets_per_cu": r64["per_cu"]},
        "nodes_accepted_per_target": round(r32["accepted"] / n_cells, 1),
        "roofline": roof(r32, "f32"),
        "roofline_fp64": roof(r64, "f64"),
    }

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        dom = P.domains[0]
        rng = np.random.default_rng(0)
        tg = np.sort(rng.choice(n_cells, min(args.cpu_sample, n_cells), replace=False))
        t0 = time.perf_counter()
        f_or, ion_or, _ = oracle.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0],
                                       f_prev=None, targets=tg)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(len(tg) * npix / dt, 1), "unit": "updates/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"{len(tg)} random targets of one sweep (tree build included), {dt:.1f} s"}
        # error of both forms against the oracle on the same sweep input (zero previous flux)
        sel = f_or > 1e-6 * f_or.max()
        for key, r in (("err_fp32c_vs_oracle", r32), ("err_fp64_vs_oracle", r64)):
            rel = np.abs(r["flux0"][tg][sel] - f_or[sel]) / f_or[sel]
            line[key] = {"max_rel": float(rel.max()), "p99_9": float(np.percentile(rel, 99.9)),
                         "cells": int(sel.sum()), "input": "absorbing sweep, zero previous flux"}

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
