"""Throughput of the TreeRay/OnTheSpot hot path on one MI355X.

A step is one outer iteration over the whole grid: point-source deposit, cell
quantities, FP64 node moments, the sweep (walk + node->ray mapping + per-ray
On-the-Spot integration + sum over rays) and delta_cell.  Inputs (densities,
previous flux) are resident in HBM before the timed region.

The default workload is the adaptive grid: 16^3 root blocks of 8^3 cells
refined twice where n_H > 1e3 over a 256^3 log-normal field (sigma 1.5),
9.9M leaf cells, 1000 sources in dense cells, N_side 4 (192 rays), theta 0.5,
64 evaluation points.  The FP32C form is timed over --steps for `value`; the
FP64 form runs the same steps on identical inputs (the same previous flux)
over --fp64-steps for the speed-up.  The FP64 CPU oracle is timed on a
bounded sample of targets on the host (all cores and one core) and gives the
error of both forms on an absorbing sweep with zero previous flux, away from
the ionisation fronts (targets with a neighbour of the other ionisation state
in the oracle are excluded and counted).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1..5]
                    [--fp64-steps K2] [--fp64-warmup W2] [--graph-steps G]
                    [--forms both|fp32c|fp64] [--no-cpu-baseline]
                    [--cpu-sample N] [--cpu-sample-1core N]
                    [--launch-fp32c W,T,B,I,A] [--launch-fp64 W,T,B,I,A] [--autotune]
                    [--n-src N] [--copy-mib M] [--theta T] [--theta-if T] [--theta-src T]
                    [--per-domain K]

--launch-* fix the sweep's launch shape (waves per target, targets per CU,
buffer 1 = LDS / 2 = device memory, integration 1 = a lane per ray / 2 = a
wave per ray / 3, 4, 5 = groups of at least 4, 8, 16 lanes per ray, 6, 7, 8
the same with the FP32 march, accumulation 1 = hardware atomics / 2 =
compare-and-swap); without them the shape the autotuner found for the
workload is used (configs 2 and 5), or searched (--autotune, other workloads);
--n-src N replaces the workload by the config-3 grid with N equal sources
(the source-count scaling); --copy-mib adds plain device copies of known
size, the calibration of the HBM byte counters in a profiled run;
--per-domain K times K sweeps of every domain of a multi-domain workload in a
context of its own, one after another, against the one batched launch.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target-cell·ray updates/s, FP32-compensated vs FP64, at ≤1e-4 rel flux err"
# MI355X published peaks
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# Algorithmic work per unit (a traversal model of the sweep):
#   per accepted node 40 FLOP per angular sub-point (s^3 of them), 80 for the
#   radial weights and 60 for the accumulation into the ray buffer;
#   per tested node its FP32 record (com 12 B, eps/alpha/E/V 16 B, topology
#   4 B) or FP64 record (60 B), read once per target (no reuse credited)
FLOP_SUBPOINT, FLOP_RADIAL, FLOP_ACCUM = 40, 80, 60
NODE_BYTES = {"f32": 32, "f64": 60}
# lanes per ray reported by the library -> the integration code of tr_set_launch
# (+3 when the rays were marched in FP32)
INT_MODE = {1: 1, 64: 2, 4: 3, 8: 4, 16: 5}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=5, help="workload 1..5")
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed steps of the FP64 form (at most --steps)")
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--graph-steps", type=int, default=1, help="hipGraph step replays timed per form")
    ap.add_argument("--forms", default="both", choices=["both", "fp32c", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536, help="oracle targets timed on all host cores")
    ap.add_argument("--cpu-sample-1core", type=int, default=1024, help="oracle targets timed on one core")
    ap.add_argument("--no-autotune", action="store_true", help="library default shape where none is tuned")
    ap.add_argument("--autotune", action="store_true", help="search the launch shape even where one is tuned")
    ap.add_argument("--launch-fp32c", default="", help="W,T,B,I,A launch shape of the FP32C sweep")
    ap.add_argument("--launch-fp64", default="", help="W,T,B,I,A launch shape of the FP64 sweep")
    ap.add_argument("--n-src", type=int, default=0, help="config-3 grid with this many equal sources")
    ap.add_argument("--copy-mib", type=int, default=0, help="plain copies of this size after the steps")
    ap.add_argument("--theta", type=float, default=None, help="override the opening angle")
    ap.add_argument("--theta-if", type=float, default=None, help="IF MAC opening angle")
    ap.add_argument("--theta-src", type=float, default=None, help="Src MAC opening angle")
    ap.add_argument("--per-domain", type=int, default=0,
                    help="also time this many sweeps of every domain in a context of its own (multi-domain workloads)")
    return ap.parse_args()


# Launch shapes (waves, targets per CU, buffer, integration, atomics) the
# autotuner picks on MI355X for the two profiled workloads; the defaults there,
# so that the committed counter summaries (taken at these shapes) apply.
TUNED_LAUNCH = {
    (5, "fp32c"): "16,1,1,6,2", (5, "fp64"): "16,1,1,3,1",
    (2, "fp32c"): "16,1,1,6,2", (2, "fp64"): "16,1,1,3,1",
}


def profile_text(name):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return fh.read()


def measured_traffic(workload, form, launch, digest):
    """HBM bytes per sweep launch from the committed counter summary, if it was
    taken from the current kernel sources and the same launch shape."""
    text = profile_text(f"k_sweep_{workload}_hbm_traffic.txt")
    if text is None:
        return None
    want = f"form={form} launch={launch} sources={digest}"
    for line in text.splitlines():
        m = re.match(r"^traffic_bytes_per_launch (\S+) (.*)$", line.strip())
        if m and m.group(2) == want:
            return int(float(m.group(1)))
    return None


def measured_counters(workload, form, launch, digest):
    """VALU issue utilisation, VALU instructions per accepted node and mean
    occupancy of the sweep from the committed counter summary, if it was taken
    from the current kernel sources and the same launch shape."""
    text = profile_text(f"k_sweep_{workload}_sq_counters.txt")
    if text is None or f"kernel sources digest: {digest}" not in text:
        return {}
    out = {}
    for line in text.splitlines():
        m = re.match(r"^counters (\S+) launch=(\S+) (.*)$", line.strip())
        if m and m.group(1) == form and m.group(2) == launch:
            for kv in m.group(3).split():
                k, v = kv.split("=")
                out[k] = float(v)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "sharding the targets over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2105_09644_amd as T
    from paper_2105_09644_amd import build as B
    from paper_2105_09644_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    T.load_library()
    digest = B.source_digest()
    P = W.source_count_problem(args.n_src) if args.n_src > 0 else W.CONFIGS[args.config]()
    for key in ("theta", "theta_if", "theta_src"):
        if getattr(args, key) is not None:
            setattr(P.params, key, getattr(args, key))
    npix = 12 * P.params.nside ** 2
    sub = P.params.subsample ** 3
    n_cells = P.total_cells()
    nh = torch.tensor(np.concatenate(P.n_h), dtype=torch.float64, device="cuda")
    props = torch.cuda.get_device_properties(0)
    waves_per_simd_max = props.max_threads_per_multi_processor // 64 // 4
    log(f"workload {P.name}: {n_cells} cells, {len(P.domains)} domain(s), N_PIX {npix}")

    # the previous flux both forms start from: one optically thin FP32C sweep
    with T.context_for(P, T.TR_FP32C) as ctx:
        f_thin = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
        ctx.build(nh, None, thin=True)
        ctx.sweep(f_thin)
        ctx.sync()
    log("previous flux: optically thin FP32C sweep")

    def run_form(prec, launch, steps, warmup, graph_steps):
        name = "fp32c" if prec == T.TR_FP32C else "fp64"
        ctx = T.context_for(P, prec)
        f_prev = f_thin.clone()
        f_new = torch.zeros_like(f_prev)
        ion = torch.zeros(n_cells, dtype=torch.uint8, device="cuda")
        ctx.build(nh, f_prev)
        if not launch and not args.autotune and args.n_src == 0:
            launch = TUNED_LAUNCH.get((args.config, name), "")
        if launch:
            ctx.set_launch(*(int(x) for x in launch.split(",")))
        elif not args.no_autotune:
            t0 = time.perf_counter()
            ctx.autotune()
            log(f"{name}: autotuned in {time.perf_counter() - t0:.1f} s")
        for _ in range(warmup):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)
            ctx.delta(f_new, f_prev)
        torch.cuda.synchronize()
        log(f"{name}: timing {steps} steps")
        sweep_ms = []
        acc = tested = guard = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.build(nh, f_prev)
            ctx.sweep(f_new, ion)        # the sweep kernel is bracketed by HIP events on its stream
            ctx.delta(f_new, f_prev)     # synchronises the stream
            st = ctx.stats()
            sweep_ms.append(st.last_sweep_ms)
            acc, tested, guard = st.nodes_accepted, st.nodes_tested, st.guard_recomputes
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = ctx.stats()
        res = dict(ms_per_step=dt * 1e3, value=n_cells * npix / dt, sweep_ms=float(np.mean(sweep_ms)),
                   steps=steps, warmup=warmup, accepted=int(acc), tested=int(tested), guard=int(guard),
                   waves=st.waves_per_target, per_cu=st.targets_per_cu, lds=st.buffer_in_lds,
                   nr=st.n_radial_max, intw=st.integration_wave, cas=st.lds_cas, int32=st.integration_fp32,
                   rays32=st.rays_fp32, rays64=st.rays_fp64_again, tab=st.nodes_tabulated, regrouped=st.rays_regrouped)
        im = INT_MODE[res["intw"]] + (3 if res["int32"] else 0)
        res["launch"] = f"{res['waves']},{res['per_cu']},{1 if res['lds'] else 2},{im},{2 if res['cas'] else 1}"
        log(f"{name}: {res['ms_per_step']:.2f} ms/step, sweep {res['sweep_ms']:.2f} ms, launch {res['launch']}")
        # the same outer iteration as one hipGraph launch, ping-ponging two flux buffers
        if graph_steps > 0:
            a, b = f_prev.clone(), f_new
            ctx.step(nh, a, b, ion)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(graph_steps):
                ctx.step(nh, a, b, ion)
                a, b = b, a
            res["ms_per_step_graph"] = (time.perf_counter() - t0) / graph_steps * 1e3
            log(f"{name}: hipGraph step {res['ms_per_step_graph']:.2f} ms")
        # parity input independent of either side: an absorbing sweep with zero previous flux
        ctx.build(nh, None)
        ctx.sweep(f_new, ion)
        ctx.sync()
        res["flux0"] = f_new.cpu().numpy()
        ctx.close()
        return res

    forms = {}
    if args.forms in ("both", "fp32c"):
        forms["f32"] = run_form(T.TR_FP32C, args.launch_fp32c, args.steps, args.warmup, args.graph_steps)
    if args.forms in ("both", "fp64"):
        k64 = args.steps if args.forms == "fp64" else max(1, min(args.fp64_steps, args.steps))
        forms["f64"] = run_form(T.TR_FP64, args.launch_fp64, k64, args.fp64_warmup, min(args.graph_steps, 1))

    per_domain = None
    if args.per_domain > 0 and len(P.domains) > 1:
        # the same sweep of the main form with every domain in a context of its
        # own, one after another, at the batched launch shape
        rf = forms["f32"] if "f32" in forms else forms["f64"]
        prec = T.TR_FP32C if "f32" in forms else T.TR_FP64
        off = np.cumsum([0] + [d.n_cells() for d in P.domains])
        kernel_ms = 0.0
        wall = 0.0
        for d in range(len(P.domains)):
            Pd = W.Problem(f"{P.name}_domain{d}", [P.domains[d]], [P.n_h[d]], [P.src_xyz[d]], [P.src_q[d]],
                           P.params)
            lo, hi = int(off[d]), int(off[d + 1])
            with T.context_for(Pd, prec) as c:
                fp = f_thin[lo:hi].clone()
                fo = torch.zeros_like(fp)
                io = torch.zeros(hi - lo, dtype=torch.uint8, device="cuda")
                c.build(nh[lo:hi].clone(), fp)
                c.set_launch(*(int(x) for x in rf["launch"].split(",")))
                c.sweep(fo, io)
                c.sync()
                ms = []
                t0 = time.perf_counter()
                for _ in range(args.per_domain):
                    c.sweep(fo, io)
                    c.sync()
                    ms.append(c.stats().last_sweep_ms)
                wall += (time.perf_counter() - t0) / args.per_domain
                kernel_ms += float(np.mean(ms))
        per_domain = {"contexts": len(P.domains), "launch": rf["launch"], "sweeps_each": args.per_domain,
                      "sweep_ms_sum": round(kernel_ms, 3), "wall_ms_sum": round(wall * 1e3, 3),
                      "batched_sweep_ms": round(rf["sweep_ms"], 3),
                      "batched_over_sequential": round(rf["sweep_ms"] / kernel_ms, 4)}
        log(f"per-domain contexts: {kernel_ms:.2f} ms of sweeps one after another against "
            f"{rf['sweep_ms']:.2f} ms batched")

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
        """The sweep kernel against the VALU and the HBM rooflines (algorithmic work)."""
        sec = r["sweep_ms"] * 1e-3
        flops = (FLOP_SUBPOINT * sub + FLOP_RADIAL + FLOP_ACCUM) * r["accepted"]
        byts = NODE_BYTES[form] * r["tested"]
        fname = "fp32c" if form == "f32" else "fp64"
        traffic = measured_traffic(P.name, fname, r["launch"], digest)
        cnt = measured_counters(P.name, fname, r["launch"], digest)
        # the instantiation that ran (buffer place 3: LDS ray buffers in passes)
        kernel = "k_sweep_cas" if r["cas"] else ("k_sweep_pass" if r["lds"] == 3 else "k_sweep")
        occ = r["per_cu"] * r["waves"] / 4.0                 # resident waves per SIMD
        alu = {"bound": "alu", "achieved": round(flops / sec / 1e12, 3), "peak": VALU_PEAK_TFLOPS[form],
               "unit": "TFLOP/s", "frac": round(flops / sec / 1e12 / VALU_PEAK_TFLOPS[form], 4),
               "traffic": traffic, "kernel": kernel, "flops_per_launch": int(flops),
               "flop_model": f"{FLOP_SUBPOINT} x {sub} sub-points + {FLOP_RADIAL + FLOP_ACCUM} per accepted node",
               "launch_ms": round(r["sweep_ms"], 3),
               "valu_issue_utilisation": cnt.get("valu_issue"),
               "valu_insts_per_accepted_node": cnt.get("valu_per_node"),
               "occupancy_waves_per_simd": occ, "occupancy_peak": waves_per_simd_max,
               "occupancy_measured": cnt.get("occupancy")}
        hbm = {"bound": "hbm", "achieved": round(byts / sec / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(byts / sec / 1e9 / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": kernel,
               "bytes_per_launch": int(byts), "byte_model": f"{NODE_BYTES[form]} B per tested node",
               "launch_ms": round(r["sweep_ms"], 3)}
        if traffic:
            hbm["measured_gbs"] = round(traffic / sec / 1e9, 1)
            hbm["measured_frac"] = round(traffic / sec / 1e9 / HBM_PEAK_GBS, 5)
        # the bound is the roofline that allows the lesser throughput
        t_alu = flops / (VALU_PEAK_TFLOPS[form] * 1e12)
        t_hbm = max(byts, traffic or 0) / (HBM_PEAK_GBS * 1e9)
        return (alu, hbm) if t_alu >= t_hbm else (hbm, alu)

    main_form = "f32" if "f32" in forms else "f64"
    r = forms[main_form]
    roof, other = roofline(r, main_form)
    line = {
        "metric": METRIC,
        "value": round(r["value"], 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": r["warmup"],
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_form,
        "data": "synthetic",
        "config": {"workload": P.name, "cells": n_cells, "domains": len(P.domains), "n_pix": npix,
                   "n_sources": int(sum(len(q) for q in P.src_q)),
                   "theta": P.params.theta, "theta_if": P.params.theta_if, "theta_src": P.params.theta_src,
                   "n_radial_max": r["nr"],
                   "precision": (("FP32 walk/weights/ray buffers, FP64 moments; FP32 ray march with compensated "
                                  "Phi and flux sums, FP64 again near ionisation fronts" if r["int32"] else
                                  "FP32 walk/weights/ray buffers, FP64 moments, ray integration and flux sums")
                                 if main_form == "f32" else "FP64 throughout")},
        "sweep_ms": round(r["sweep_ms"], 3),
        "ms_per_step_graph": round(r.get("ms_per_step_graph", float("nan")), 3),
        "launch": r["launch"],
        "nodes_accepted_per_target": round(r["accepted"] / n_cells, 1),
        "nodes_tested_per_target": round(r["tested"] / n_cells, 1),
        "guard_recomputes_per_accepted_node": round(r["guard"] / max(1, r["accepted"]), 4),
        "rays_marched_fp32": r["rays32"], "rays_marched_again_fp64": r["rays64"], "rays_regrouped": r["regrouped"],
        "nodes_from_angular_table": round(r["tab"] / max(1, r["accepted"]), 4),
        "roofline": roof,
        "roofline_other": other,
    }
    if "f32" in forms and "f64" in forms:
        r64 = forms["f64"]
        a64, h64 = roofline(r64, "f64")
        line["fp64"] = {"value": round(r64["value"], 1), "steps": r64["steps"], "warmup": r64["warmup"],
                        "ms_per_step": round(r64["ms_per_step"], 3), "sweep_ms": round(r64["sweep_ms"], 3),
                        "launch": r64["launch"], "roofline": a64, "roofline_other": h64}
        line["speedup_vs_fp64"] = round(r["value"] / r64["value"], 3)
        line["sweep_speedup_vs_fp64"] = round(r64["sweep_ms"] / r["sweep_ms"], 3)

    if per_domain:
        line["per_domain"] = per_domain
    if not args.no_cpu_baseline:
        line.update(cpu_baseline(args, P, forms, npix, W))

    print(json.dumps(line), flush=True)


def cpu_baseline(args, P, forms, npix, W):
    """The FP64 oracle on a bounded sample of targets: seeded random cells with
    their 26 neighbours, so that cells next to an ionisation front can be told
    apart; half of the centres are drawn among the cells the GPU's FP64 (else
    FP32C) sweep finds lit, half uniformly.  Timed on all host cores and on one
    core; the tree build is timed on its own."""
    import oracle
    oracle.build(force=False)
    out = {}
    ref = forms["f64"]["flux0"] if "f64" in forms else forms["f32"]["flux0"]
    rng = np.random.default_rng([2105, 9644, 77])
    per_dom = []       # (domain index, cell offset, centres, targets)
    off = 0
    n_cells = P.total_cells()
    want = args.cpu_sample
    for d, dom in enumerate(P.domains):
        n = dom.n_cells()
        share = max(1, int(round(want * n / n_cells / 27)))
        lit = np.nonzero(ref[off:off + n] > 0)[0]
        c_lit = rng.choice(lit, size=min(share // 2, lit.size), replace=False) if lit.size else np.zeros(0, int)
        c_any = rng.choice(n, size=min(share - c_lit.size, n), replace=False)
        centres = np.unique(np.concatenate([c_lit, c_any]))
        nb = W.cell_neighbours(dom, centres)
        tg = np.unique(np.concatenate([centres, nb[nb >= 0]]))
        per_dom.append((d, off, centres, nb, tg))
        off += n
    n_tg = sum(x[4].size for x in per_dom)
    log(f"oracle: {n_tg} targets ({sum(x[2].size for x in per_dom)} centres with their neighbours) "
        f"on {oracle.num_threads()} threads")
    f_or = {}
    t_all = 0.0
    for d, o, centres, nb, tg in per_dom:
        dom = P.domains[d]
        tm = []
        f, _, _ = oracle.sweep(dom, P.params, P.n_h[d], P.src_xyz[d], P.src_q[d], f_prev=None, targets=tg,
                               timing=tm)
        t_all += tm[0]
        f_or[d] = dict(zip(tg.tolist(), f.tolist()))
    threads = oracle.num_threads()
    # one core, on the first targets of the first domain's sample
    d, o, centres, nb, tg = per_dom[0]
    tg1 = tg[:min(args.cpu_sample_1core, tg.size)]
    tm = []
    oracle.sweep(P.domains[d], P.params, P.n_h[d], P.src_xyz[d], P.src_q[d], f_prev=None, targets=tg1,
                 threads=1, timing=tm)
    t_one = tm[0]
    out["cpu_baseline"] = {
        "value": round(n_tg * npix / t_all, 1), "unit": "updates/s", "cores": threads, "kind": "oracle",
        "sample": f"{n_tg} targets of one absorbing sweep with zero previous flux (seeded cells and their "
                  f"26 neighbours), {t_all:.1f} s of target loop (tree builds excluded)",
        "cpu": cpu_model(),
        "one_core": {"value": round(tg1.size * npix / t_one, 1), "unit": "updates/s", "cores": 1,
                     "sample": f"{tg1.size} of those targets, {t_one:.1f} s"},
    }
    log(f"oracle: {n_tg * npix / t_all:.3e} updates/s on {threads} threads, "
        f"{tg1.size * npix / t_one:.3e} on one")
    # error of each form against the oracle, away from the fronts
    for form, rr in forms.items():
        rel_all, flags_bad, excluded, lit_n = [], 0, 0, 0
        fmax = max(max(v.values()) for v in f_or.values())
        for d, o, centres, nb, tg in per_dom:
            fo = f_or[d]
            for i, c in enumerate(centres.tolist()):
                ion_c = fo[c] > 0
                near = any((fo[j] > 0) != ion_c for j in nb[i].tolist() if j >= 0)
                if near:
                    excluded += 1
                    continue
                g = rr["flux0"][o + c]
                if (g > 0) != ion_c:
                    flags_bad += 1
                if fo[c] > 1e-6 * fmax:
                    lit_n += 1
                    rel_all.append(abs(g - fo[c]) / fo[c])
        rel = np.asarray(rel_all) if rel_all else np.zeros(1)
        out["err_fp32c_vs_oracle" if form == "f32" else "err_fp64_vs_oracle"] = {
            "max_rel": float(rel.max()), "p99_9": float(np.percentile(rel, 99.9)),
            "cells": lit_n, "front_excluded": excluded, "flag_mismatches": flags_bad,
            "input": "absorbing sweep, zero previous flux; centres within one cell of the oracle's front excluded"}
    return out


if __name__ == "__main__":
    main()
