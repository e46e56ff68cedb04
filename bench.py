"""Throughput of the TreeRay/OnTheSpot hot path on one MI355X.

A step is one outer iteration over the whole grid: point-source deposit,
cell quantities, FP64 node moments, the sweep (walk + node->ray mapping +
per-ray On-the-Spot integration + sum over rays) and delta_cell.  Inputs
(densities, previous flux) are resident in HBM before the timed region.

The default workload is the uniform 64^3 grid around one Q = 1e49 source
with N_side 4 (192 rays), theta 0.5 and 48 evaluation points.  The FP32C form
(FP32 walk, weights and ray buffers; FP64 moments, integration and flux sums)
is timed for `value`; the FP64 form runs the same steps on
the same inputs for the speed-up.  The FP64 CPU oracle is timed on a bounded
sample of targets on the host and gives the reported error of both forms.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--config 1..5] [--forms both|fp32c|fp64]
                    [--launch-fp32c W,T,B,I,A] [--launch-fp64 W,T,B,I,A] [--copy-mib M]
                    [--theta T] [--theta-if T] [--theta-src T]

--launch-* fix the sweep's launch shape (waves per target, targets per CU,
buffer 1 = LDS / 2 = device memory, integration 1 = a lane per ray / 2 = a
wave per ray / 3, 4, 5 = a group of 4, 8, 16 lanes per ray, accumulation
1 = hardware atomics / 2 = compare-and-swap) instead of autotuning it; --copy-mib
adds plain device copies of known size, the calibration of the HBM byte
counters in a profiled run.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target-cell·ray updates/s, FP32-compensated vs FP64, at ≤1e-4 rel flux err"
HBM_PEAK_GBS = 8000.0
# Vector peak without packed FP32 math (which this build disables):
# 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz; the FP64 vector peak is the same.
VALU_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
# Algorithmic work per unit (the derivation is itemised in the design notes):
#   bytes: every tested node's record (geometry + moments) is read once per
#          target, 32 B in FP32, 60 B in FP64; per target 8 B flux + 1 B flag
#   flops: opening test 11 per tested node; 56 per angular sub-point (s^3 per
#          accepted node); 240 per accepted node for the radial weights and the
#          accumulation; 20 per (ray, evaluation point) of the integration;
#          2 per ray and 30 per target for the sum over rays and the self term
NODE_BYTES = {"f32": 32, "f64": 60}
TARGET_BYTES = 9
# lanes per ray reported by the library -> the integration code of tr_set_launch
INT_MODE = {1: 1, 64: 2, 4: 3, 8: 4, 16: 5}
FLOP_TEST, FLOP_SUB, FLOP_NODE, FLOP_POINT, FLOP_RAY, FLOP_TARGET = 11, 56, 240, 20, 2, 30
SRC_FILES = ["csrc/treeray.hip", "csrc/kernels.h", "csrc/tr_internal.h", "csrc/topology.cpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="workload 1..5")
    ap.add_argument("--forms", default="both", choices=["both", "fp32c", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=98304, help="oracle targets in the CPU baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch-fp32c", default="", help="W,T,B,I,A launch shape of the FP32C sweep")
    ap.add_argument("--launch-fp64", default="", help="W,T,B,I,A launch shape of the FP64 sweep")
    ap.add_argument("--copy-mib", type=int, default=0, help="plain copies of this size after the steps")
    ap.add_argument("--theta", type=float, default=None, help="override the opening angle")
    ap.add_argument("--theta-if", type=float, default=None, help="IF MAC opening angle")
    ap.add_argument("--theta-src", type=float, default=None, help="Src MAC opening angle")
    return ap.parse_args()


def source_digest():
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, "paper_2105_09644_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, form, launch):
    """HBM bytes per sweep launch from the committed counter summary, if it was
    taken from the current kernel sources and the same launch shape."""
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    want = f"form={form} launch={launch} sources={source_digest()}"
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^traffic_bytes_per_launch (\S+) (.*)$", line.strip())
            if m and m.group(2) == want:
                return int(float(m.group(1)))
    return None


def measured_valu_issue(workload, form, launch):
    """The sweep's VALU issue utilisation (wave instructions per CU per clock) from the
    committed issue-counter summary, if it was taken from the current kernel sources
    and the same launch shape."""
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_sq_counters.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    if f"kernel sources digest: {source_digest()}" not in text:
        return None
    m = re.search(("--launch-fp32c" if form == "fp32c" else "--launch-fp64") + r" (\S+)", text)
    if not m or m.group(1) != launch:
        return None
    sec = re.search(r"^" + form + r" \(.*?(?:\n\n|\Z)", text, re.S | re.M)
    u = re.search(r"VALU issue utilisation: .*= ([0-9.]+)", sec.group(0)) if sec else None
    return float(u.group(1)) if u else None


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
    for key in ("theta", "theta_if", "theta_src"):
        if getattr(args, key) is not None:
            setattr(P.params, key, getattr(args, key))
    npix = 12 * P.params.nside ** 2
    sub = P.params.subsample ** 3
    n_cells = P.total_cells()
    nh = torch.tensor(np.concatenate(P.n_h), dtype=torch.float64, device="cuda")
    log(f"workload {P.name}: {n_cells} cells, {len(P.domains)} domain(s), N_PIX {npix}")

    def run_form(prec, launch):
        name = "fp32c" if prec == T.TR_FP32C else "fp64"
        ctx = T.context_for(P, prec)
        f_prev = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
        f_new = torch.zeros_like(f_prev)
        ion = torch.zeros(n_cells, dtype=torch.uint8, device="cuda")
        ctx.build(nh, None, thin=True)
        ctx.sweep(f_prev, ion)
        ctx.build(nh, f_prev)
        if launch:
            ctx.set_launch(*(int(x) for x in launch.split(",")))
        elif not args.no_autotune:
            ctx.autotune()
        for _ in range(args.warmup):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)
            ctx.delta(f_new, f_prev)
        torch.cuda.synchronize()
        log(f"{name}: timing {args.steps} steps")
        sweep_ms = []
        acc = tested = 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)        # the sweep kernel is bracketed by HIP events on its stream
            ctx.delta(f_new, f_prev)     # synchronises the stream
            st = ctx.stats()
            sweep_ms.append(st.last_sweep_ms)
            acc, tested = st.nodes_accepted, st.nodes_tested
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = ctx.stats()
        res = dict(ms_per_step=dt * 1e3, value=n_cells * npix / dt, sweep_ms=float(np.mean(sweep_ms)),
                   accepted=int(acc), tested=int(tested), waves=st.waves_per_target,
                   per_cu=st.targets_per_cu, lds=st.buffer_in_lds, guard=int(st.guard_recomputes),
                   nr=st.n_radial_max, intw=st.integration_wave, cas=st.lds_cas)
        res["launch"] = (f"{res['waves']},{res['per_cu']},{1 if res['lds'] else 2},{INT_MODE[res['intw']]},"
                         f"{2 if res['cas'] else 1}")
        log(f"{name}: {res['ms_per_step']:.2f} ms/step, sweep {res['sweep_ms']:.2f} ms, launch {res['launch']}")
        # the same outer iteration as one hipGraph launch, ping-ponging two flux buffers
        a, b = f_prev.clone(), f_new
        ctx.step(nh, a, b, ion)
        ctx.step(nh, b, a, ion)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.step(nh, a, b, ion)
            a, b = b, a
        res["ms_per_step_graph"] = (time.perf_counter() - t0) / args.steps * 1e3
        # parity input independent of either side: an absorbing sweep with zero previous flux
        ctx.build(nh, None)
        ctx.sweep(f_new, ion)
        ctx.sync()
        res["flux0"] = f_new.cpu().numpy()
        ctx.close()
        return res

    forms = {}
    if args.forms in ("both", "fp32c"):
        forms["f32"] = run_form(T.TR_FP32C, args.launch_fp32c)
    if args.forms in ("both", "fp64"):
        forms["f64"] = run_form(T.TR_FP64, args.launch_fp64)

    if args.copy_mib > 0:
        # calibration for the HBM byte counters: plain copies of known size
        n = args.copy_mib * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.copy_mib} MiB read + written")

    def roofline(r, form):
        """The sweep kernel against the VALU and the HBM rooflines."""
        sec = r["sweep_ms"] * 1e-3
        flops = (FLOP_TEST * r["tested"] + (FLOP_SUB * sub + FLOP_NODE) * r["accepted"]
                 + n_cells * npix * (FLOP_POINT * r["nr"] + FLOP_RAY) + FLOP_TARGET * n_cells)
        byts = NODE_BYTES[form] * r["tested"] + TARGET_BYTES * n_cells
        tf = flops / sec / 1e12
        gbs = byts / sec / 1e9
        traffic = measured_traffic(P.name, "fp32c" if form == "f32" else "fp64", r["launch"])
        kernel = "k_sweep_cas" if r["cas"] else "k_sweep"   # the instantiation that ran
        issue = measured_valu_issue(P.name, "fp32c" if form == "f32" else "fp64", r["launch"])
        # the bound is the roofline that allows the lesser throughput
        t_alu = flops / (VALU_PEAK_TFLOPS[form] * 1e12)
        t_hbm = byts / (HBM_PEAK_GBS * 1e9)
        alu = {"bound": "alu", "achieved": round(tf, 3), "peak": VALU_PEAK_TFLOPS[form], "unit": "TFLOP/s",
               "frac": round(tf / VALU_PEAK_TFLOPS[form], 4), "traffic": traffic, "kernel": kernel,
               "flops_per_launch": int(flops), "launch_ms": round(r["sweep_ms"], 3),
               "valu_issue_utilisation": issue}
        hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": kernel,
               "bytes_per_launch": int(byts), "launch_ms": round(r["sweep_ms"], 3)}
        return (alu, hbm) if t_alu >= t_hbm else (hbm, alu)

    main_form = "f32" if "f32" in forms else "f64"
    r = forms[main_form]
    roof, other = roofline(r, main_form)
    line = {
        "metric": METRIC,
        "value": round(r["value"], 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_form,
        "data": "synthetic",
        "config": {"workload": P.name, "cells": n_cells, "domains": len(P.domains), "n_pix": npix,
                   "theta": P.params.theta, "theta_if": P.params.theta_if, "theta_src": P.params.theta_src,
                   "n_radial_max": r["nr"],
                   "precision": ("FP32 walk/weights/ray buffers, FP64 moments, ray integration and flux sums"
                                 if main_form == "f32" else "FP64 throughout")},
        "sweep_ms": round(r["sweep_ms"], 3),
        "ms_per_step_graph": round(r["ms_per_step_graph"], 3),
        "launch": r["launch"],
        "nodes_accepted_per_target": round(r["accepted"] / n_cells, 1),
        "nodes_tested_per_target": round(r["tested"] / n_cells, 1),
        "roofline": roof,
        "roofline_other": other,
    }
    if "f32" in forms and "f64" in forms:
        r64 = forms["f64"]
        a64, h64 = roofline(r64, "f64")
        line["fp64"] = {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 3),
                        "sweep_ms": round(r64["sweep_ms"], 3), "launch": r64["launch"],
                        "roofline": a64, "roofline_other": h64}
        line["speedup_vs_fp64"] = round(r["value"] / r64["value"], 3)

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        rng = np.random.default_rng(0)
        tg = np.sort(rng.choice(n_cells, min(args.cpu_sample, n_cells), replace=False))
        log(f"oracle: {len(tg)} targets on the host")
        f_or = np.empty(len(tg))
        t0 = time.perf_counter()
        off = 0
        for d, dom in enumerate(P.domains):
            n = dom.n_cells()
            sel = (tg >= off) & (tg < off + n)
            if sel.any():
                f, _, _ = oracle.sweep(dom, P.params, P.n_h[d], P.src_xyz[d], P.src_q[d],
                                       f_prev=None, targets=tg[sel] - off)
                f_or[sel] = f
            off += n
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(len(tg) * npix / dt, 1), "unit": "updates/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"{len(tg)} random targets of one absorbing sweep "
                                          f"(tree builds included), {dt:.1f} s"}
        # error of the forms against the oracle on the same sweep input (zero previous flux)
        sel = f_or > 1e-6 * f_or.max()
        for form, rr in forms.items():
            rel = np.abs(rr["flux0"][tg][sel] - f_or[sel]) / f_or[sel]
            line["err_fp32c_vs_oracle" if form == "f32" else "err_fp64_vs_oracle"] = {
                "max_rel": float(rel.max()), "p99_9": float(np.percentile(rel, 99.9)),
                "cells": int(sel.sum()), "input": "absorbing sweep, zero previous flux"}

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
