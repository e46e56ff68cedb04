"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Both sides get the same seeded inputs and, for absorbing sweeps, the same
previous flux (the oracle's own thin sweep), so every sweep is compared
element by element.  Tolerances:

* FP64 form: |F_gpu - F_or| <= 1e-10 F_or on every cell with
  F_or > 1e-6 max F_or, and identical ionisation flags.
* FP32C form: the same relative error bounded by 1e-4 on cells that are not
  within one cell of the oracle's ionisation front (cells next to a dark
  cell); ionisation flags identical away from the front.  Near the front the
  flux is a small difference of large terms and the FP32 mapping error is
  amplified; those cells are counted and reported, not bounded.
"""
import math
import sys

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.fixture(scope="module")
def T():
    import paper_2105_09644_amd as T
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    T.load_library()
    return T


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_sweep(T, P, prec, f_prev=None, thin=False, targets=None, launch=None, **over):
    ctx = T.context_for(P, prec, **over)
    if launch is not None:
        ctx.set_launch(*launch)
    n = ctx.n_cells
    nh = torch.tensor(np.concatenate(P.n_h), dtype=torch.float64, device="cuda")
    fp = None if f_prev is None else torch.tensor(f_prev, dtype=torch.float64, device="cuda")
    ctx.build(nh, fp, thin=thin)
    if targets is None:
        out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        ion = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        ctx.sweep(out, ion)
    else:
        tg = torch.tensor(targets, dtype=torch.int64, device="cuda")
        out = torch.full((len(targets),), -1.0, dtype=torch.float64, device="cuda")
        ion = torch.full((len(targets),), 7, dtype=torch.uint8, device="cuda")
        ctx.sweep_targets(tg, out, ion)
    ctx.sync()
    st = ctx.stats()
    res = out.cpu().numpy(), ion.cpu().numpy(), st
    ctx.close()
    return res


def orc_sweep(orc, P, f_prev=None, thin=False, targets=None, **over):
    """Oracle per domain; targets are global cell indices."""
    outs, ions = [], []
    off = 0
    fp_all = f_prev
    for d, dom in enumerate(P.domains):
        n = dom.n_cells()
        fp = None if fp_all is None else fp_all[off:off + n]
        tg = None
        if targets is not None:
            sel = (targets >= off) & (targets < off + n)
            tg = targets[sel] - off
        kw = dict(over)
        if thin:
            kw["alpha_b"] = 0.0
        if tg is None or len(tg):
            f, ion, _ = orc.sweep(dom, P.params, P.n_h[d], P.src_xyz[d], P.src_q[d], f_prev=fp, targets=tg, **kw)
            outs.append(f)
            ions.append(ion)
        off += n
    return np.concatenate(outs), np.concatenate(ions)


def front_mask(P, f_or):
    """Cells within one cell (26-neighbourhood) of a dark cell; uniform grids only."""
    masks = []
    off = 0
    for dom in P.domains:
        n = dom.n_cells()
        f = f_or[off:off + n]
        if dom.leaf_blocks is not None:
            masks.append(f <= 0)
            off += n
            continue
        e = dom.extent_finest()
        dark = (f <= 0).reshape(e)
        near = np.zeros_like(dark)
        pad = np.pad(dark, 1, constant_values=False)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    near |= pad[1 + dx:1 + dx + e[0], 1 + dy:1 + dy + e[1], 1 + dz:1 + dz + e[2]]
        masks.append(near.ravel())
        off += n
    return np.concatenate(masks)


def compare(f_gpu, ion_gpu, f_or, ion_or, tol, front=None, name=""):
    assert np.all(np.isfinite(f_gpu)), f"{name}: non-finite GPU flux"
    sel = f_or > 1e-6 * f_or.max()
    if front is not None:
        sel &= ~front
    rel = np.abs(f_gpu[sel] - f_or[sel]) / f_or[sel]
    log(f"{name}: cells {sel.sum()} max rel {rel.max():.3e} p99.9 {np.percentile(rel, 99.9):.3e} "
        f"L1 {np.sum(np.abs(f_gpu[sel] - f_or[sel])) / np.sum(f_or[sel]):.3e}")
    assert rel.max() <= tol, f"{name}: max relative error {rel.max():.3e} > {tol}"
    ion_sel = np.ones_like(ion_or, bool) if front is None else ~front
    bad = np.count_nonzero(ion_gpu[ion_sel] != ion_or[ion_sel])
    assert bad == 0, f"{name}: {bad} ionisation flags differ"


def cases():
    return {
        "uniform16": lambda: W.small_uniform(16, n_radial=20),
        "lognormal16": lambda: W.small_lognormal(16, n_src=3, seed=1),
        "padded24": lambda: W.small_lognormal(24, n_src=2, seed=2, nside=1),
        "amr": lambda: W.small_amr(2, seed=3),
        "nside4": lambda: W.small_lognormal(16, n_src=2, seed=4, nside=4, n_radial=24),
    }


@pytest.mark.parametrize("case", list(cases()))
def test_fp64_sweeps(T, orc, case):
    P = cases()[case]()
    log(f"case {case}: cells {P.total_cells()}")
    f0, i0 = orc_sweep(orc, P, thin=True)
    g0, j0, st = gpu_sweep(T, P, T.TR_FP64, thin=True)
    compare(g0, j0, f0, i0, TOL64, name=f"{case} thin fp64")
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    g1, j1, st = gpu_sweep(T, P, T.TR_FP64, f_prev=f0)
    compare(g1, j1, f1, i1, TOL64, name=f"{case} absorbing fp64")
    assert st.overflow == 0


@pytest.mark.parametrize("case", list(cases()))
def test_fp32c_sweeps(T, orc, case):
    P = cases()[case]()
    f0, i0 = orc_sweep(orc, P, thin=True)
    g0, j0, st = gpu_sweep(T, P, T.TR_FP32C, thin=True)
    compare(g0, j0, f0, i0, TOL32, name=f"{case} thin fp32c")
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    g1, j1, st = gpu_sweep(T, P, T.TR_FP32C, f_prev=f0)
    compare(g1, j1, f1, i1, TOL32, front=front_mask(P, f1), name=f"{case} absorbing fp32c")
    log(f"  guard recomputes {st.guard_recomputes} of {st.nodes_accepted * 64} sub-points")


def test_batched_domains(T, orc):
    # two domains of different sizes in one context: one launch covers both
    A = W.small_lognormal(16, n_src=2, seed=5)
    B = W.small_lognormal(24, n_src=1, seed=6)
    P = W.Problem("two", A.domains + B.domains, A.n_h + B.n_h, A.src_xyz + B.src_xyz, A.src_q + B.src_q, A.params)
    f0, i0 = orc_sweep(orc, P, thin=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
        g1, j1, st = gpu_sweep(T, P, prec, f_prev=f0)
        compare(g1, j1, f1, i1, tol, front=None if prec == T.TR_FP64 else front_mask(P, f1),
                name=f"batched prec {prec}")


def test_target_list_and_ragged_tail(T, orc):
    P = W.small_lognormal(16, n_src=3, seed=7)
    f0, _ = orc_sweep(orc, P, thin=True)
    rng = np.random.default_rng(3)
    tg = rng.choice(P.total_cells(), 1237, replace=False)   # not a multiple of any launch width
    f1, i1 = orc_sweep(orc, P, f_prev=f0, targets=tg)
    g1, j1, _ = gpu_sweep(T, P, T.TR_FP64, f_prev=f0, targets=tg)
    compare(g1, j1, f1, i1, TOL64, name="target list")
    g2, j2, _ = gpu_sweep(T, P, T.TR_FP64, f_prev=f0, targets=np.zeros(0, np.int64))
    assert len(g2) == 0


def test_config1_fp64_full(T, orc):
    P = W.config1()
    log("config1: 32^3, N_side 2, 32 points")
    f0, i0 = orc_sweep(orc, P, thin=True)
    g0, j0, _ = gpu_sweep(T, P, T.TR_FP64, thin=True)
    compare(g0, j0, f0, i0, TOL64, name="config1 thin fp64")
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    g1, j1, _ = gpu_sweep(T, P, T.TR_FP64, f_prev=f0)
    compare(g1, j1, f1, i1, TOL64, name="config1 absorbing fp64")


def test_delta_matches_oracle(T, orc):
    P = W.small_lognormal(16, n_src=3, seed=8)
    f0, _ = orc_sweep(orc, P, thin=True)
    f1, _ = orc_sweep(orc, P, f_prev=f0)
    ctx = T.context_for(P, T.TR_FP64)
    a = torch.tensor(f1, device="cuda")
    b = torch.tensor(f0, device="cuda")
    d = ctx.delta(a, b)
    assert d[0] == pytest.approx(orc.delta_cell(f1, f0), rel=1e-14)
    # median of a field with many zeros, and the zero-normaliser case
    z = f0.copy()
    z[: len(z) // 2 + 3] = 0.0
    d = ctx.delta(torch.tensor(f1, device="cuda"), torch.tensor(z, device="cuda"))
    assert math.isinf(d[0]) and math.isinf(orc.delta_cell(f1, z))
    ctx.close()


def test_solve_matches_oracle(T, orc):
    # the same fixed number of outer iterations on both sides
    P = W.small_lognormal(16, n_src=2, seed=9)
    P.params.max_iter = 3
    P.params.eps_lim = 0.0
    dom = P.domains[0]
    f_or, ion_or, it, dl = orc.solve(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], eps_lim=0.0, max_iter=3)
    ctx = T.context_for(P, T.TR_FP64)
    nh = torch.tensor(P.n_h[0], device="cuda")
    out = torch.zeros(ctx.n_cells, dtype=torch.float64, device="cuda")
    ion = torch.zeros(ctx.n_cells, dtype=torch.uint8, device="cuda")
    iters, delta = ctx.solve(nh, out, ion, allow_noconv=True)
    assert iters == it == 3
    assert delta == pytest.approx(dl, rel=1e-6)
    compare(out.cpu().numpy(), ion.cpu().numpy(), f_or, ion_or, 1e-9, name="solve x3 fp64")
    ctx.close()


def test_graph_step_replays(T, orc):
    """tr_step (one outer iteration captured as a hipGraph) against the eager
    build/sweep/delta calls, replayed several times with eager work between
    the replays, every replay checked; then against the oracle."""
    P = W.small_lognormal(16, n_src=3, seed=10)
    f0, _ = orc_sweep(orc, P, thin=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    d_or = orc.delta_cell(f1, f0)
    # atomic accumulation order differs between launches: FP64 agrees to
    # rounding, FP32C to its own tolerance away from the front
    for prec, tol in ((T.TR_FP64, 1e-12), (T.TR_FP32C, TOL32)):
        ctx = T.context_for(P, prec)
        n = ctx.n_cells
        nh = torch.tensor(P.n_h[0], device="cuda")
        fp = torch.tensor(f0, device="cuda")
        ref = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.build(nh, fp)
        ctx.sweep(ref)
        d_ref = ctx.delta(ref, fp)
        ref_h = ref.cpu().numpy()
        ref_ion = (ref_h > 0).astype(np.uint8)
        fr = None if prec == T.TR_FP64 else front_mask(P, ref_h)
        out = torch.zeros(n, dtype=torch.float64, device="cuda")
        ion = torch.zeros(n, dtype=torch.uint8, device="cuda")
        scratch = torch.zeros(n, dtype=torch.float64, device="cuda")
        for rep in range(4):
            out.fill_(-1.0)
            ion.fill_(7)
            d = ctx.step(nh, fp, out, ion)
            g = out.cpu().numpy()
            log(f"graph prec {prec} replay {rep}: delta {d[0]:.6e} eager {d_ref[0]:.6e}")
            compare(g, ion.cpu().numpy(), ref_h, ref_ion, tol, front=fr, name=f"replay {rep} vs eager")
            assert d[0] == pytest.approx(d_ref[0], rel=1e-9 if prec == T.TR_FP64 else 1e-3)
            # eager work between replays: another build and sweep, a torch kernel
            ctx.build(nh, thin=True)
            ctx.sweep(scratch)
            scratch.mul_(0.5)
            torch.cuda.synchronize()
        tol_or = TOL64 if prec == T.TR_FP64 else TOL32
        compare(out.cpu().numpy(), ion.cpu().numpy(), f1, i1, tol_or,
                front=None if prec == T.TR_FP64 else front_mask(P, f1), name=f"graph step prec {prec}")
        assert d[0] == pytest.approx(d_or, rel=1e-9 if prec == T.TR_FP64 else 1e-3)
        # new buffers: the graph is captured again
        out2 = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.step(nh, fp, out2)
        assert torch.equal(out2 > 0, out > 0)
        with pytest.raises(T.TreeRayError) as e:
            ctx.step(nh, fp, fp)
        assert e.value.status == T.TR_EINVAL
        ctx.close()


def test_graph_after_scratch_regrowth(T, orc):
    """A captured step graph refers to the sweep's scratch memory (the overflow
    queue, ray-buffer slabs).  A target list longer than the grid regrows that
    scratch; the next step must capture again instead of replaying the old
    graph.  theta = 0.05 sends every walk through the overflow queue."""
    P = W.small_lognormal(16, n_src=2, seed=25)
    f0, _ = orc_sweep(orc, P, thin=True, theta=0.05)
    f1, i1 = orc_sweep(orc, P, f_prev=f0, theta=0.05)
    ctx = T.context_for(P, T.TR_FP64, theta=0.05)
    ctx.set_launch(4, 0, 2, 0, 0)
    n = ctx.n_cells
    nh = torch.tensor(P.n_h[0], device="cuda")
    fp = torch.tensor(f0, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.step(nh, fp, out)
    compare(out.cpu().numpy(), (out > 0).cpu().numpy().astype(np.uint8), f1, i1, TOL64, name="step before regrowth")
    # 3 n targets (every cell three times): the overflow queue and slabs grow
    tg = torch.arange(3 * n, dtype=torch.int64, device="cuda") % n
    ft = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    ctx.build(nh, fp)
    ctx.sweep_targets(tg, ft)
    ctx.sync()
    assert ctx.stats().overflow == 0
    compare(ft.cpu().numpy()[:n], (ft[:n] > 0).cpu().numpy().astype(np.uint8), f1, i1, TOL64, name="long list")
    out.fill_(-1.0)
    ctx.step(nh, fp, out)
    ctx.sync()
    assert ctx.stats().overflow == 0
    compare(out.cpu().numpy(), (out > 0).cpu().numpy().astype(np.uint8), f1, i1, TOL64, name="step after regrowth")
    ctx.close()


@pytest.mark.parametrize("theta_if,theta_src", [(0.25, 0.2), (1e-6, 1e-6)])
def test_if_and_src_macs(T, orc, theta_if, theta_src):
    """IF MAC and Src MAC (Sec. 2.4) against the oracle, on a previous flux that
    holds an ionisation front (the oracle's absorbing sweep)."""
    P = W.small_lognormal(16, n_src=2, seed=23)
    f0, _ = orc_sweep(orc, P, thin=True)
    f1, _ = orc_sweep(orc, P, f_prev=f0)
    over = dict(theta_if=theta_if, theta_src=theta_src)
    f2, i2 = orc_sweep(orc, P, f_prev=f1, **over)
    for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
        g2, j2, st = gpu_sweep(T, P, prec, f_prev=f1, **over)
        compare(g2, j2, f2, i2, tol, front=None if prec == T.TR_FP64 else front_mask(P, f2),
                name=f"macs {theta_if}/{theta_src} prec {prec}")
        log(f"  accepted per target {st.nodes_accepted / P.total_cells():.1f}")
    # thin, emission resolved to cells
    t0, k0 = orc_sweep(orc, P, thin=True, theta_src=1e-6)
    g0, j0, _ = gpu_sweep(T, P, T.TR_FP64, thin=True, theta_src=1e-6)
    compare(g0, j0, t0, k0, TOL64, name="thin src mac fp64")


def test_long_walks_use_device_lists(T, orc):
    # theta = 0.05 on 16^3 accepts nearly every cell: the walk lists exceed
    # the LDS capacity and every target goes through the device-memory pass
    P = W.small_lognormal(16, n_src=2, seed=25)
    f0, i0 = orc_sweep(orc, P, thin=True, theta=0.05)
    for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
        g0, j0, st = gpu_sweep(T, P, prec, thin=True, theta=0.05)
        compare(g0, j0, f0, i0, tol, name=f"theta 0.05 prec {prec}")
        assert st.overflow == 0
        assert st.nodes_accepted / P.total_cells() > 2048


def test_few_targets_with_long_walks(T, orc):
    # a short target list whose walks all overflow the LDS lists, with ray
    # buffers in device memory (FP64, FP32C), split (FP32C at N_side 4 with
    # 64 points) or in LDS in passes over the rays (FP64 at N_side 4): the
    # second pass runs more workgroups than the first, each with its own
    # buffer slab
    rng = np.random.default_rng(26)
    # (at 16 waves the next target is walked by four waves, here with device lists)
    cases = [(W.small_lognormal(16, n_src=2, seed=25), T.TR_FP64, 2, 0, 4),
             (W.small_lognormal(16, n_src=2, seed=25), T.TR_FP32C, 2, 0, 4),
             (W.small_lognormal(16, n_src=2, seed=25), T.TR_FP32C, 1, 1, 16),
             (W.small_lognormal(16, n_src=2, seed=27, nside=4, n_radial=64), T.TR_FP32C, 1, 2, 4),
             (W.small_lognormal(16, n_src=2, seed=27, nside=4, n_radial=64), T.TR_FP64, 1, 3, 4),
             (W.small_lognormal(16, n_src=2, seed=27, nside=4, n_radial=64), T.TR_FP64, 1, 3, 16)]
    for P, prec, buf, where, waves in cases:
        tg = np.sort(rng.choice(P.total_cells(), 37, replace=False))
        f0, i0 = orc_sweep(orc, P, thin=True, targets=tg, theta=0.05)
        g0, j0, st = gpu_sweep(T, P, prec, thin=True, targets=tg, launch=(waves, 0, buf, 0, 0), theta=0.05)
        assert st.overflow == 0 and st.buffer_in_lds == where
        assert st.nodes_accepted / len(tg) > 2048
        compare(g0, j0, f0, i0, TOL64 if prec == T.TR_FP64 else TOL32,
                name=f"37 targets prec {prec} buffer {buf} waves {waves}")


@pytest.mark.parametrize("radius_cells", [0.45, 1.7])
def test_sphere_sources(T, orc, radius_cells):
    """Sources as uniform spheres (Sec. 2.7): the exact-volume deposit against
    the oracle's, through thin and absorbing sweeps, uniform and AMR grids."""
    for P in (W.small_lognormal(16, n_src=4, seed=26), W.small_amr(2, seed=27)):
        r = radius_cells * P.domains[0].finest_dx_cm()
        f0, i0 = orc_sweep(orc, P, thin=True, src_radius_cm=r)
        f1, i1 = orc_sweep(orc, P, f_prev=f0, src_radius_cm=r)
        for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
            g0, j0, _ = gpu_sweep(T, P, prec, thin=True, src_radius_cm=r)
            compare(g0, j0, f0, i0, tol, name=f"{P.name} r {radius_cells} thin prec {prec}")
            g1, j1, _ = gpu_sweep(T, P, prec, f_prev=f0, src_radius_cm=r)
            compare(g1, j1, f1, i1, tol, front=None if prec == T.TR_FP64 else front_mask(P, f1),
                    name=f"{P.name} r {radius_cells} absorbing prec {prec}")


@pytest.mark.parametrize("eps_kernel,mass_kernel", [(1, 0), (2, 0), (4, 0), (5, 0), (6, 6), (3, 6)])
def test_radial_kernel_variants(T, orc, eps_kernel, mass_kernel):
    """Radial kernels of App. A (W_f,1, W_f,2, N-point W_f,3, W_p and W_g for the
    emission; W_g for A, E, V) against the oracle."""
    P = W.small_lognormal(16, n_src=3, seed=32, nside=2)
    over = dict(eps_kernel=eps_kernel, mass_kernel=mass_kernel)
    f0, i0 = orc_sweep(orc, P, thin=True, **over)
    f1, i1 = orc_sweep(orc, P, f_prev=f0, **over)
    for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
        g0, j0, _ = gpu_sweep(T, P, prec, thin=True, **over)
        compare(g0, j0, f0, i0, tol, name=f"kernels {eps_kernel}/{mass_kernel} thin prec {prec}")
        g1, j1, _ = gpu_sweep(T, P, prec, f_prev=f0, **over)
        compare(g1, j1, f1, i1, tol, front=None if prec == T.TR_FP64 else front_mask(P, f1),
                name=f"kernels {eps_kernel}/{mass_kernel} absorbing prec {prec}")


@pytest.mark.parametrize("make", [lambda: W.small_lognormal(16, n_src=3, seed=43),
                                  lambda: W.small_lognormal(24, n_src=2, seed=44, nside=1),
                                  lambda: W.rabbit_hole(0.5, 48, 2, nside=2)], ids=["cube16", "padded24", "slab48"])
def test_periodic_boundaries(T, orc, make):
    """Periodic boundaries (Sec. 2.8, nearest copy of every node) against the oracle."""
    P = make()
    f0, i0 = orc_sweep(orc, P, thin=True, periodic=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0, periodic=True)
    for prec, tol in ((T.TR_FP64, TOL64), (T.TR_FP32C, TOL32)):
        g0, j0, _ = gpu_sweep(T, P, prec, thin=True, periodic=True)
        compare(g0, j0, f0, i0, tol, name=f"{P.name} periodic thin prec {prec}")
        g1, j1, _ = gpu_sweep(T, P, prec, f_prev=f0, periodic=True)
        compare(g1, j1, f1, i1, tol, front=None if prec == T.TR_FP64 else front_mask(P, f1),
                name=f"{P.name} periodic absorbing prec {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_launch_shapes(T, orc, prec):
    # every integration form (a lane, a wave, a group of 4, 8 or 16 lanes per
    # ray), both buffer places, 1, 4 and 16 waves per target and both
    # accumulation forms give the oracle's flux; 60 sources on 12 rays put more
    # emitting points on a ray than a group of 4 or 8 lanes holds, so the
    # wider groups run too
    P = W.small_lognormal(16, n_src=60, seed=7, nside=1, n_radial=24)
    f0, i0 = orc_sweep(orc, P, thin=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    pr, tol = (T.TR_FP64, TOL64) if prec == "fp64" else (T.TR_FP32C, TOL32)
    front = None if prec == "fp64" else front_mask(P, f1)
    shapes = [(w, b, im, 0) for w in (1, 4, 16) for b in (1, 2) for im in (1, 2, 3, 4, 5, 6, 7, 8)]
    shapes += [(w, 1, 0, am) for w in (8, 16) for am in (1, 2)]   # the accumulation forms
    for waves, buf, im, am in shapes:
        name = f"shape waves {waves} buffer {buf} integration {im} atomics {am}"
        g0, j0, st = gpu_sweep(T, P, pr, thin=True, launch=(waves, 0, buf, im, am))
        assert (st.waves_per_target, st.buffer_in_lds) == (waves, int(buf == 1))
        if im:
            assert st.integration_wave == {1: 1, 2: 64, 3: 4, 4: 8, 5: 16, 6: 4, 7: 8, 8: 16}[im]
            # the FP32 march exists for FP32 buffers; the FP64 form takes the FP64 groups
            assert st.integration_fp32 == int(im >= 6 and prec == "fp32c")
        cas = prec == "fp32c" and buf == 1 and waves in (8, 16) and am != 1
        assert st.lds_cas == int(cas)
        compare(g0, j0, f0, i0, tol, name=name + " thin")
        g1, j1, _ = gpu_sweep(T, P, pr, f_prev=f0, launch=(waves, 0, buf, im, am))
        compare(g1, j1, f1, i1, tol, front=front, name=name + " absorbing")


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_many_emitting_points(T, orc, prec):
    # 4000 sources in 16^3 cells, 12 rays of 120 points, theta 0.3: rays hold
    # from one to more than 64 emitting points, so the rays beyond a group of
    # 4 or 16 lanes are marched again by groups of 8 to 64 lanes, and those
    # beyond 64 points by a wave
    P = W.small_lognormal(16, n_src=4000, seed=11, nside=1, n_radial=120, theta=0.3)
    f0, i0 = orc_sweep(orc, P, thin=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    pr, tol = (T.TR_FP64, TOL64) if prec == "fp64" else (T.TR_FP32C, TOL32)
    front = None if prec == "fp64" else front_mask(P, f1)
    for im in ((3, 5) if prec == "fp64" else (3, 6, 8)):
        for waves in (4, 16):
            name = f"{prec} many emitters waves {waves} integration {im}"
            g0, j0, st = gpu_sweep(T, P, pr, thin=True, launch=(waves, 0, 0, im, 0))
            log(f"{name}: rays regrouped {st.rays_regrouped}, in FP32 {st.rays_fp32}")
            assert st.rays_regrouped > 0
            compare(g0, j0, f0, i0, tol, name=name + " thin")
            g1, j1, _ = gpu_sweep(T, P, pr, f_prev=f0, launch=(waves, 0, 0, im, 0))
            compare(g1, j1, f1, i1, tol, front=front, name=name + " absorbing")


@pytest.mark.parametrize("waves", [4, 16])
def test_split_ray_buffers(T, orc, waves):
    # N_side 4 with 64 radial points: four rows per ray (197 KB) do not fit in
    # LDS, three do, so the FP32C sweep keeps A, E, V in LDS and the emission
    # rows in device memory; the FP64 sweep maps and integrates the rays in
    # passes with LDS buffers, or keeps everything in device memory
    P = W.small_lognormal(16, n_src=6, seed=8, nside=4, n_radial=64)
    f0, i0 = orc_sweep(orc, P, thin=True)
    f1, i1 = orc_sweep(orc, P, f_prev=f0)
    front = front_mask(P, f1)
    for im in (0, 1, 2, 8):
        name = f"split waves {waves} integration {im}"
        g0, j0, st = gpu_sweep(T, P, T.TR_FP32C, thin=True, launch=(waves, 0, 0, im, 0))
        assert st.buffer_in_lds == 2
        compare(g0, j0, f0, i0, TOL32, name=name + " thin")
        g1, j1, _ = gpu_sweep(T, P, T.TR_FP32C, f_prev=f0, launch=(waves, 0, 0, im, 0))
        compare(g1, j1, f1, i1, TOL32, front=front, name=name + " absorbing")
    # FP64: four rows per ray in LDS for a third of the rays at a time (passes),
    # or all rows in device memory
    for buf, where in ((0, 3), (2, 0)):
        for im in (0, 1, 2):
            g1, j1, st = gpu_sweep(T, P, T.TR_FP64, f_prev=f0, launch=(waves, 0, buf, im, 0))
            assert st.buffer_in_lds == where
            compare(g1, j1, f1, i1, TOL64, name=f"fp64 waves {waves} buffer {buf} integration {im}")


@pytest.mark.parametrize("make", [lambda: W.small_lognormal(16, n_src=6, seed=31, nside=4, n_radial=48),
                                  lambda: W.small_amr(2, seed=32, n_src=12),
                                  lambda: W.small_uniform(24, q=2e48, n_radial=40)])
def test_fp32_march_across_fronts(T, orc, make):
    """The FP32 ray march (integration 6-8) on absorbing sweeps that hold
    ionisation fronts: zero previous flux (zeta_d = 2) and the oracle's own
    thin flux.  Away from the front the flux agrees with the FP64 oracle to
    1e-4 and the flags agree; some rays must have gone back to FP64 (a source
    below 1e-2 of its emitted Phi) and most must have stayed in FP32."""
    P = make()
    f0, _ = orc_sweep(orc, P, thin=True)
    for fp in (None, f0):
        f1, i1 = orc_sweep(orc, P, f_prev=fp)
        front = front_mask(P, f1)
        for im in (6, 7, 8):
            g1, j1, st = gpu_sweep(T, P, T.TR_FP32C, f_prev=fp, launch=(0, 0, 0, im, 0))
            assert st.integration_fp32 == 1
            log(f"{P.name} prev {'zero' if fp is None else 'thin'} integration {im}: rays in FP32 {st.rays_fp32}, "
                f"again in FP64 {st.rays_fp64_again}, front cells {int(front.sum())}")
            assert st.rays_fp32 > 0 and st.rays_fp64_again < st.rays_fp32
            compare(g1, j1, f1, i1, TOL32, front=front, name=f"fp32 march {im}")
        if fp is None:
            assert st.rays_fp64_again > 0


def test_errors(T):
    P = W.small_uniform(16)
    ctx = T.context_for(P, T.TR_FP64)
    nh = torch.tensor(P.n_h[0], device="cuda")
    bad = nh.clone()
    bad[5] = float("nan")
    with pytest.raises(T.TreeRayError) as e:
        ctx.build(bad)
    assert e.value.status == T.TR_EINVAL
    bad[5] = -1.0
    with pytest.raises(T.TreeRayError):
        ctx.build(bad)
    with pytest.raises(T.TreeRayError) as e:
        ctx.set_sources(0, [[1e30, 0, 0]], [1e48])
    assert e.value.status == T.TR_EINVAL
    out = torch.zeros(ctx.n_cells, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TreeRayError) as e:   # sweep before a successful build
        ctx.sweep(out)
    assert e.value.status == T.TR_ESTATE
    ctx.build(nh, thin=True)
    tg = torch.tensor([0, 5, ctx.n_cells + 3], dtype=torch.int64, device="cuda")
    o = torch.zeros(3, dtype=torch.float64, device="cuda")
    ctx.sweep_targets(tg, o)
    with pytest.raises(T.TreeRayError) as e:
        ctx.sync()
    assert e.value.status == T.TR_EINVAL
    assert math.isnan(o[2].item()) and o[0].item() > 0
    # launch options out of range
    for bad_launch in ((3, 0, 0, 0, 0), (4, -1, 0, 0, 0), (4, 0, 3, 0, 0), (4, 0, 0, 9, 0), (4, 0, 0, 0, 3)):
        with pytest.raises(T.TreeRayError) as e:
            ctx.set_launch(*bad_launch)
        assert e.value.status == T.TR_EINVAL
    ctx.close()


def test_many_ray_passes(T, orc):
    # N_side 8 with 64 points in FP64: 768 rays of four rows (1.6 MB) are
    # mapped and integrated in passes of a few dozen rays held in LDS
    P = W.small_lognormal(16, n_src=3, seed=44, nside=8, n_radial=64)
    rng = np.random.default_rng(45)
    tg = np.sort(rng.choice(P.total_cells(), 96, replace=False))
    f0, i0 = orc_sweep(orc, P, thin=True, targets=tg)
    f1, i1 = orc_sweep(orc, P, f_prev=None, targets=tg)
    for waves in (4, 16):
        g0, j0, st = gpu_sweep(T, P, T.TR_FP64, thin=True, targets=tg, launch=(waves, 0, 1, 0, 0))
        assert st.buffer_in_lds == 3
        compare(g0, j0, f0, i0, TOL64, name=f"N_side 8 passes waves {waves} thin")
        g1, j1, _ = gpu_sweep(T, P, T.TR_FP64, targets=tg, launch=(waves, 0, 1, 0, 0))
        compare(g1, j1, f1, i1, TOL64, name=f"N_side 8 passes waves {waves} absorbing")
