"""Seeded synthetic inputs for the TreeRay/OnTheSpot sweep.

This module only *describes* problems: grids (uniform or block-structured
adaptive), hydrogen number densities, point sources and run parameters.  It
holds none of the method's arithmetic (no tree, no rays, no kernels), so both
the HIP library and the FP64 CPU oracle can be fed from it.

Grid description (shared by every consumer):

* A domain is an array of ``nroot`` root blocks of 8^3 cells each, of side
  ``root_block_cm``.  Blocks may be refined up to ``max_level`` times; a block
  at level L has side ``root_block_cm / 2**L``.
* ``leaf_blocks is None``: uniform grid (``max_level == 0``); cells are in
  global C order over (x, y, z), z fastest -- the order of ``n_h.ravel()``
  for an ``n_h[x, y, z]`` array.
* otherwise ``leaf_blocks`` is an int32 array ``[n, 4] = (level, bi, bj, bk)``
  with (bi, bj, bk) the block index at that level; cells are ordered block by
  block, C order (x slowest, z fastest) inside each block.

Physical setup (Sec. 3.1 of the paper for the constants): pure hydrogen,
alpha_B = 2.7e-13 cm^3 s^-1 (Case B at 1e4 K), cubic boxes of side 4 pc with
isolated boundaries.  Random streams use ``numpy.random.default_rng`` seeded
with ``[2105, 9644, k]`` (config k) or ``[2105, 9644, 4, m]`` (domain m of
the batched config).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PC_CM = 3.0856775814913673e18
ALPHA_B = 2.7e-13          # cm^3 s^-1, Case-B recombination coefficient at 1e4 K
HNU_EUV_ERG = 13.6 * 1.602176634e-12   # mean EUV photon energy used to report e
C_LIGHT = 2.99792458e10
BOX_PC = 4.0
BLOCK = 8


@dataclass
class Domain:
    nroot: tuple                      # root blocks per axis
    root_block_cm: float              # side of one root block
    max_level: int = 0                # refinement levels above the root level
    leaf_blocks: Optional[np.ndarray] = None   # int32 [n,4] (level, bi, bj, bk)

    def n_cells(self) -> int:
        if self.leaf_blocks is None:
            return int(np.prod(self.nroot)) * BLOCK ** 3
        return int(self.leaf_blocks.shape[0]) * BLOCK ** 3

    def finest_dx_cm(self) -> float:
        return self.root_block_cm / (BLOCK * 2 ** self.max_level)

    def extent_finest(self) -> tuple:
        f = BLOCK * 2 ** self.max_level
        return tuple(int(n) * f for n in self.nroot)


@dataclass
class Params:
    nside: int = 2
    n_radial: int = 0         # >0: that many evaluation points; 0: from eta_r
    eta_r: float = 2.0
    theta: float = 0.5
    alpha_b: float = ALPHA_B
    subsample: int = 4
    zeta_g: bool = True
    eps_lim: float = 1e-2
    max_iter: int = 30
    theta_if: float = 0.0     # IF MAC opening angle; <= 0: off
    theta_src: float = 0.0    # Src MAC opening angle; <= 0: off
    src_radius_cm: float = 0.0   # > 0: sources are uniform spheres of this radius
    eps_kernel: int = 0       # emission kernel: 0 two-point W_f,3, 1 W_f,1, 2 W_f,2, 3 W_f,3, 4 N-point W_f,3, 5 W_p, 6 W_g
    mass_kernel: int = 0      # kernel of A, E, V: 0 or 5 W_p, 6 W_g
    periodic: bool = False    # periodic boundaries (nearest copy of every node)


@dataclass
class Problem:
    name: str
    domains: List[Domain]
    n_h: List[np.ndarray]              # per domain, float64 [n_cells]
    src_xyz: List[np.ndarray]          # per domain, float64 [n_src, 3] in cm
    src_q: List[np.ndarray]            # per domain, float64 [n_src] photons/s
    params: Params = field(default_factory=Params)

    def total_cells(self) -> int:
        return sum(d.n_cells() for d in self.domains)


def rng_for(*key) -> np.random.Generator:
    return np.random.default_rng([2105, 9644, *key])


def uniform_domain(n: int, box_pc: float = BOX_PC) -> Domain:
    if n % BLOCK:
        raise ValueError("grid size must be a multiple of 8")
    nb = n // BLOCK
    return Domain(nroot=(nb, nb, nb), root_block_cm=box_pc * PC_CM / nb)


def lognormal_field(n: int, sigma: float, mean: float, rng: np.random.Generator) -> np.ndarray:
    """Log-normal density with a P(k) ~ k^-4 Gaussian random field underneath.

    Steps: white noise in C order, amplitude |k|^-2 in Fourier space (integer
    wavenumbers, k = 0 removed), back-transform, standardise, exponentiate with
    ``sigma`` and rescale to the exact empirical ``mean``.
    """
    g0 = rng.standard_normal((n, n, n))
    gk = np.fft.rfftn(g0)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / k2[nz]
    g = np.fft.irfftn(gk * amp, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    rho = np.exp(sigma * g)
    return rho * (mean / rho.mean())


def uniform_sources(rng: np.random.Generator, n_src: int, box_cm: float,
                    logq_lo: float, logq_hi: float):
    xyz = rng.uniform(0.0, box_cm, size=(n_src, 3))
    q = 10.0 ** rng.uniform(logq_lo, logq_hi, size=n_src)
    return xyz, q


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def config1(thin: bool = False) -> Problem:
    """Uniform 32^3, n_H = 100, Q = 1e48 at the box centre, N_side 2, 32 points."""
    n = 32
    dom = uniform_domain(n)
    box = BOX_PC * PC_CM
    p = Params(nside=2, n_radial=32, theta=0.5, alpha_b=0.0 if thin else ALPHA_B)
    return Problem("uniform32_q1e48_nside2", [dom], [np.full(n ** 3, 100.0)],
                   [np.array([[box / 2, box / 2, box / 2]])], [np.array([1e48])], p)


def config2() -> Problem:
    """Uniform 64^3, n_H = 100, Q = 1e49 at the box centre, N_side 4, 48 points."""
    n = 64
    dom = uniform_domain(n)
    box = BOX_PC * PC_CM
    p = Params(nside=4, n_radial=48, theta=0.5)
    return Problem("uniform64_q1e49_nside4", [dom], [np.full(n ** 3, 100.0)],
                   [np.array([[box / 2, box / 2, box / 2]])], [np.array([1e49])], p)


def config3(n: int = 128) -> Problem:
    """128^3 log-normal (sigma 1, mean 100), 16 sources, Q in [1e47, 1e50], N_PIX 48."""
    rng = rng_for(3)
    dom = uniform_domain(n)
    nh = lognormal_field(n, 1.0, 100.0, rng).ravel()
    xyz, q = uniform_sources(rng, 16, BOX_PC * PC_CM, 47.0, 50.0)
    p = Params(nside=2, n_radial=0, eta_r=2.0, theta=0.5)
    return Problem(f"lognormal{n}_16src_nside2", [dom], [nh], [xyz], [q], p)


def source_count_problem(n_src: int, n: int = 128, q_total: float = 1.6e50) -> Problem:
    """The config-3 grid (128^3 log-normal, sigma 1) with ``n_src`` sources at
    seeded uniform-random positions sharing the total rate ``q_total`` equally:
    the input of the source-count scaling (Sec. 5.2 measures 10 to 10^4 sources)."""
    rng = rng_for(3)
    dom = uniform_domain(n)
    nh = lognormal_field(n, 1.0, 100.0, rng).ravel()
    srng = rng_for(52, n_src)
    xyz = srng.uniform(0.0, BOX_PC * PC_CM, size=(n_src, 3))
    q = np.full(n_src, q_total / n_src)
    p = Params(nside=2, n_radial=0, eta_r=2.0, theta=0.5)
    return Problem(f"lognormal{n}_{n_src}src_equal_nside2", [dom], [nh], [xyz], [q], p)


def config4(n_domains: int = 64, sizes=(32, 48, 64, 96)) -> Problem:
    """64 independent log-normal domains of uneven sizes, 1-8 sources each, N_PIX 48."""
    doms, nhs, xyzs, qs = [], [], [], []
    for m in range(n_domains):
        rng = rng_for(4, m)
        n = int(rng.choice(np.asarray(sizes)))
        dom = uniform_domain(n)
        nh = lognormal_field(n, 1.0, 100.0, rng).ravel()
        ns = int(rng.integers(1, 9))
        xyz, q = uniform_sources(rng, ns, BOX_PC * PC_CM, 47.0, 50.0)
        doms.append(dom); nhs.append(nh); xyzs.append(xyz); qs.append(q)
    p = Params(nside=2, n_radial=0, eta_r=2.0, theta=0.5)
    return Problem(f"batched{n_domains}_lognormal_nside2", doms, nhs, xyzs, qs, p)


def amr_from_field(field: np.ndarray, nroot: int, max_level: int, threshold: float,
                   root_block_cm: float):
    """Block-structured AMR grid over a fine field.

    ``field`` is given at level 1 (twice the root-level resolution).  Level-0
    cells take the volume average of their 2^3 field cells, level-1 cells the
    field value, level-2 cells the value of their parent field cell.  A block
    is refined when the maximum of the field over its footprint exceeds
    ``threshold``.  Leaf blocks are listed depth first (root blocks in C
    order, children in (x, y, z) bit order, x the highest bit).
    """
    nf = field.shape[0]
    assert nf == nroot * BLOCK * 2
    blocks = []
    values = []

    def footprint(level, bi, bj, bk):
        # field cells covered by the block
        s = BLOCK * 2 // (2 ** level) if level <= 1 else None
        if level <= 1:
            return field[bi * s:(bi + 1) * s, bj * s:(bj + 1) * s, bk * s:(bk + 1) * s]
        # level-2 block: 8 level-2 cells = 4 field cells per axis
        s2 = BLOCK // 2
        return field[bi * s2:(bi + 1) * s2, bj * s2:(bj + 1) * s2, bk * s2:(bk + 1) * s2]

    def cells(level, bi, bj, bk):
        fp = footprint(level, bi, bj, bk)
        if level == 0:
            return fp.reshape(BLOCK, 2, BLOCK, 2, BLOCK, 2).mean(axis=(1, 3, 5))
        if level == 1:
            return fp
        return np.repeat(np.repeat(np.repeat(fp, 2, 0), 2, 1), 2, 2)

    def visit(level, bi, bj, bk):
        fp = footprint(level, bi, bj, bk)
        if level < max_level and fp.max() > threshold:
            for c in range(8):
                cx, cy, cz = (c >> 2) & 1, (c >> 1) & 1, c & 1
                visit(level + 1, 2 * bi + cx, 2 * bj + cy, 2 * bk + cz)
        else:
            blocks.append((level, bi, bj, bk))
            values.append(cells(level, bi, bj, bk).ravel())

    for bi in range(nroot):
        for bj in range(nroot):
            for bk in range(nroot):
                visit(0, bi, bj, bk)
    dom = Domain(nroot=(nroot, nroot, nroot), root_block_cm=root_block_cm,
                 max_level=max_level, leaf_blocks=np.asarray(blocks, dtype=np.int32))
    return dom, np.concatenate(values)


def config5(nroot: int = 16, n_sources: int = 1000) -> Problem:
    """Adaptive grid: 128^3 base (16^3 root blocks), two refinement levels where
    n_H > 1e3 on a 256^3 log-normal field (sigma 1.5, mean 100); sources at the
    centres of distinct finest-level cells with n_H > 1e3, Q in [1e46, 1e49];
    N_side 4, 64 points."""
    rng = rng_for(5)
    nf = nroot * BLOCK * 2
    field_ = lognormal_field(nf, 1.5, 100.0, rng)
    box = BOX_PC * PC_CM
    dom, nh = amr_from_field(field_, nroot, 2, 1e3, box / nroot)
    # finest-level dense cells
    lb = dom.leaf_blocks
    lev = np.repeat(lb[:, 0], BLOCK ** 3)
    cand = np.nonzero((lev == 2) & (nh > 1e3))[0]
    pick = rng.choice(cand, size=min(n_sources, cand.size), replace=False)
    dxf = dom.finest_dx_cm()
    a = np.arange(BLOCK)
    ci, cj, ck = np.meshgrid(a, a, a, indexing="ij")
    off = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)   # C order in block
    blk = pick // BLOCK ** 3
    loc = pick % BLOCK ** 3
    ijk = lb[blk, 1:4].astype(np.int64) * BLOCK + off[loc]        # level-2 cell index
    xyz = (ijk + 0.5) * dxf
    q = 10.0 ** rng.uniform(46.0, 49.0, size=pick.size)
    p = Params(nside=4, n_radial=64, theta=0.5)
    return Problem("amr256_s1.5_1000src_nside4", [dom], [nh], [xyz], [q], p)


def small_uniform(n: int, n_h: float = 100.0, q: float = 1e48, nside: int = 2,
                  n_radial: int = 0, theta: float = 0.5, centre: bool = True,
                  seed: int = 0) -> Problem:
    """Small uniform box (side 4 pc) with one source; for tests."""
    dom = uniform_domain(n)
    box = BOX_PC * PC_CM
    if centre:
        xyz = np.array([[box / 2, box / 2, box / 2]])
    else:
        xyz = rng_for(99, seed).uniform(0, box, size=(1, 3))
    p = Params(nside=nside, n_radial=n_radial, theta=theta)
    return Problem(f"uniform{n}", [dom], [np.full(n ** 3, n_h)], [xyz], [np.array([q])], p)


def small_lognormal(n: int, n_src: int = 3, sigma: float = 1.0, nside: int = 2,
                    theta: float = 0.5, n_radial: int = 0, seed: int = 0) -> Problem:
    """Small log-normal box with random sources; for parity tests."""
    rng = rng_for(98, seed)
    dom = uniform_domain(n)
    nh = lognormal_field(n, sigma, 100.0, rng).ravel()
    xyz, q = uniform_sources(rng, n_src, BOX_PC * PC_CM, 47.0, 50.0)
    p = Params(nside=nside, n_radial=n_radial, theta=theta)
    return Problem(f"lognormal{n}_{n_src}src", [dom], [nh], [xyz], [q], p)


def small_amr(nroot: int = 2, seed: int = 0, threshold: float = 150.0,
              n_src: int = 3, nside: int = 2) -> Problem:
    """Small two-level adaptive grid; for tests."""
    rng = rng_for(97, seed)
    nf = nroot * BLOCK * 2
    f = lognormal_field(nf, 1.0, 100.0, rng)
    box = BOX_PC * PC_CM
    dom, nh = amr_from_field(f, nroot, 2, threshold, box / nroot)
    xyz, q = uniform_sources(rng, n_src, box, 47.0, 49.0)
    p = Params(nside=nside, n_radial=24, theta=0.5)
    return Problem(f"amr{nroot}_{seed}", [dom], [nh], [xyz], [q], p)


# --------------------------------------------------------------------------
# Static radiation-only set-ups of the paper's accuracy tests (Sec. 3)
# --------------------------------------------------------------------------

M_P = 1.67262192e-24          # proton mass, g
X_H = 0.70                    # hydrogen mass fraction of the paper's gas (Sec. 3.1)


def hydrogen_density(rho_g_cm3: float) -> float:
    """n_H of gas with mass density rho and hydrogen mass fraction X_H."""
    return X_H * rho_g_cm3 / M_P


def cell_lo_size(dom: Domain):
    """Lower corner (finest-cell units, int64 [n, 3]) and size (finest cells,
    int64 [n]) of every leaf cell in the library's cell order."""
    if dom.leaf_blocks is None:
        e = dom.extent_finest()
        ix, iy, iz = np.meshgrid(*[np.arange(e[a], dtype=np.int64) for a in range(3)], indexing="ij")
        lo = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
        return lo, np.ones(lo.shape[0], np.int64)
    lb = np.asarray(dom.leaf_blocks, dtype=np.int64)
    csz = (1 << (dom.max_level - lb[:, 0]))                       # cell size of each block, finest cells
    a = np.arange(BLOCK, dtype=np.int64)
    ci, cj, ck = np.meshgrid(a, a, a, indexing="ij")
    off = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)   # C order inside a block
    lo = (lb[:, None, 1:4] * BLOCK + off[None, :, :]) * csz[:, None, None]
    return lo.reshape(-1, 3), np.repeat(csz, BLOCK ** 3)


def locate_cells(dom: Domain, pts: np.ndarray) -> np.ndarray:
    """Leaf cell (library order) containing each point given in finest-cell
    units ([m, 3], points strictly inside cells); -1 outside the domain."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    e = np.asarray(dom.extent_finest(), dtype=np.float64)
    inside = np.all((pts >= 0) & (pts < e), axis=1)
    out = np.full(pts.shape[0], -1, np.int64)
    if dom.leaf_blocks is None:
        q = np.floor(pts[inside]).astype(np.int64)
        n = np.asarray(dom.extent_finest(), dtype=np.int64)
        out[inside] = (q[:, 0] * n[1] + q[:, 1]) * n[2] + q[:, 2]
        return out
    lb = np.asarray(dom.leaf_blocks, dtype=np.int64)
    L = dom.max_level
    idx = np.nonzero(inside)[0]
    for lev in range(L + 1):
        if idx.size == 0:
            break
        sel = lb[:, 0] == lev
        if not sel.any():
            continue
        bsz = BLOCK << (L - lev)                                   # block side, finest cells
        nb = np.asarray(dom.nroot, dtype=np.int64) << lev          # blocks per axis at this level
        bno = np.nonzero(sel)[0]
        keys = (lb[bno, 1] * nb[1] + lb[bno, 2]) * nb[2] + lb[bno, 3]
        order = np.argsort(keys)
        keys, bno = keys[order], bno[order]
        b = np.floor(pts[idx] / bsz).astype(np.int64)
        k = (b[:, 0] * nb[1] + b[:, 1]) * nb[2] + b[:, 2]
        j = np.clip(np.searchsorted(keys, k), 0, keys.size - 1)
        hit = keys[j] == k
        if hit.any():
            blk = bno[j[hit]]
            csz = 1 << (L - lev)
            c = np.floor((pts[idx[hit]] - b[hit] * bsz) / csz).astype(np.int64)
            out[idx[hit]] = blk * BLOCK ** 3 + (c[:, 0] * BLOCK + c[:, 1]) * BLOCK + c[:, 2]
        idx = idx[~hit]
    return out


def cell_neighbours(dom: Domain, cells: np.ndarray) -> np.ndarray:
    """The 26 neighbours of each listed cell ([m, 26], library order, -1
    outside the domain): the leaf cells holding the points half a finest cell
    beyond each face, edge and corner of the cell.  On an adaptive grid a
    neighbour finer than the cell is the one touching that face/edge/corner's
    centre."""
    lo, size = cell_lo_size(dom)
    cells = np.asarray(cells, dtype=np.int64)
    c = lo[cells] + 0.5 * size[cells, None]
    h = 0.5 * size[cells, None] + 0.5
    dirs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
                     if (i, j, k) != (0, 0, 0)], dtype=np.float64)
    pts = c[:, None, :] + h[:, None, :] * dirs[None, :, :]
    return locate_cells(dom, pts.reshape(-1, 3)).reshape(cells.size, 26)


def sample_with_neighbours(dom: Domain, n_centres: int, rng: np.random.Generator, lit=None):
    """Seeded test sample of one domain: centre cells and their 26 neighbours.

    ``lit`` (optional bool per cell, e.g. a previous sweep's F > 0) steers the
    draw towards ionisation fronts: a third of the centres are lit cells with
    an unlit neighbour, a third lit cells, the rest uniform over the domain.
    Returns (centres [m], neighbours [m, 26] with -1 outside, targets = the
    sorted union of both)."""
    n = dom.n_cells()
    picks = []
    if lit is not None and lit.any():
        lit_idx = np.nonzero(lit)[0]
        cand = lit_idx if lit_idx.size <= 200_000 else rng.choice(lit_idx, 200_000, replace=False)
        nb = cell_neighbours(dom, cand)
        edge = cand[np.any((nb >= 0) & ~lit[np.maximum(nb, 0)], axis=1)]
        k = n_centres // 3
        if edge.size:
            picks.append(rng.choice(edge, min(k, edge.size), replace=False))
        picks.append(rng.choice(lit_idx, min(k, lit_idx.size), replace=False))
    rest = n_centres - sum(p.size for p in picks)
    picks.append(rng.choice(n, min(max(rest, 0), n), replace=False))
    centres = np.unique(np.concatenate(picks)).astype(np.int64)
    nbs = cell_neighbours(dom, centres)
    targets = np.unique(np.concatenate([centres, nbs[nbs >= 0]])).astype(np.int64)
    return centres, nbs, targets


def cell_centres_pc(dom: Domain, origin_pc=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Centres (pc) of a uniform domain's cells in the library's cell order."""
    e = dom.extent_finest()
    dx = dom.finest_dx_cm() / PC_CM
    axes = [origin_pc[a] + (np.arange(e[a]) + 0.5) * dx for a in range(3)]
    x, y, z = np.meshgrid(*axes, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def two_source_cloud(n: int = 128, nside: int = 2, theta: float = 0.5, theta_if: float = 0.0,
                     theta_src: float = 0.0) -> Problem:
    """Cloud irradiated by two sources (Sec. 3.4): the domain spans
    [-2, 4] x [-2, 4] x [-3, 3] pc; a cloud of radius 0.5 pc and density
    2.6e-21 g/cm^3 at the origin in gas of 1e-24 g/cm^3; two sources of
    3.2e48 photons/s at (-2, 0, 0) and (0, -2, 0) pc, on the domain's faces.
    The set-up is symmetric about the plane x = y."""
    dom = uniform_domain(n, box_pc=6.0)
    origin = (-2.0, -2.0, -3.0)
    c = cell_centres_pc(dom, origin)
    r2 = np.sum(c ** 2, axis=1)
    nh = np.where(r2 < 0.5 ** 2, hydrogen_density(2.6e-21), hydrogen_density(1e-24))
    src_pc = np.array([[-2.0, 0.0, 0.0], [0.0, -2.0, 0.0]])
    xyz = (src_pc - np.array(origin)) * PC_CM
    p = Params(nside=nside, n_radial=0, eta_r=2.0, theta=theta, theta_if=theta_if, theta_src=theta_src)
    return Problem(f"two_source_cloud{n}", [dom], [nh], [xyz], [np.array([3.2e48, 3.2e48])], p)


def two_source_pair(n: int = 128, sep_pc: float = 0.4, nside: int = 2, theta: float = 0.5) -> Problem:
    """The kernel-comparison variant of the two-source set-up (App. A): the
    same domain filled with rarefied gas only (1e-24 g/cm^3), sources of
    3.2e48 photons/s at (-sep, 0, 0) and (0, -sep, 0) pc."""
    dom = uniform_domain(n, box_pc=6.0)
    origin = (-2.0, -2.0, -3.0)
    nh = np.full(dom.n_cells(), hydrogen_density(1e-24))
    src_pc = np.array([[-sep_pc, 0.0, 0.0], [0.0, -sep_pc, 0.0]])
    xyz = (src_pc - np.array(origin)) * PC_CM
    p = Params(nside=nside, n_radial=0, eta_r=2.0, theta=theta)
    return Problem(f"two_source_pair{n}", [dom], [nh], [xyz], [np.array([3.2e48, 3.2e48])], p)


def rabbit_hole(width_pc: float, n_long: int = 384, axis: int = 0, nside: int = 4, theta: float = 0.25,
                theta_if: float = 0.0, theta_src: float = 0.0) -> Problem:
    """Rabbit hole (Sec. 3.2.1): a 6 x 2 x 2 pc box of cold dense gas
    (1e-18 g/cm^3) pierced along its long axis by a hole of square cross-section
    width_pc filled with warm rarefied gas (1e-24 g/cm^3); a source of 1e49
    photons/s at the hole's entrance, the centre of one 2 x 2 pc face.  The long
    axis is x (axis 0) or z (axis 2); cells are cubes, n_long along it."""
    nb = n_long // BLOCK
    nroot = [nb // 3] * 3
    nroot[axis] = nb
    dom = Domain(nroot=tuple(nroot), root_block_cm=6.0 * PC_CM / nb)
    e = dom.extent_finest()
    dx = dom.finest_dx_cm() / PC_CM
    origin = [-1.0, -1.0, -1.0]
    origin[axis] = 0.0
    axes = [origin[a] + (np.arange(e[a]) + 0.5) * dx for a in range(3)]
    g = np.meshgrid(*axes, indexing="ij")
    inside = np.ones(g[0].shape, bool)
    for a in range(3):
        if a != axis:
            inside &= np.abs(g[a]) < 0.5 * width_pc
    nh = np.where(inside, hydrogen_density(1e-24), hydrogen_density(1e-18)).ravel()
    xyz = (np.zeros(3) - np.array(origin)) * PC_CM
    p = Params(nside=nside, n_radial=0, eta_r=2.0, theta=theta, theta_if=theta_if, theta_src=theta_src)
    return Problem(f"rabbit_hole_w{width_pc:g}_axis{axis}", [dom], [nh], [xyz[None, :]], [np.array([1e49])], p)


def prev_flux_field(problem: Problem, seed: int = 0, dark_fraction: float = 0.2,
                    sigma: float = 1.0) -> np.ndarray:
    """Synthetic previous-iteration flux for every cell of ``problem``, an input
    that both sides of a parity test take: log-normal values (sigma in ln) on
    the scale of the total source rate spread over a sphere of a quarter of
    the first domain's side, with a random ``dark_fraction`` of cells at zero.
    Photons cm^-2 s^-1, float64, domains concatenated."""
    rng = rng_for(96, seed)
    n = problem.total_cells()
    side = problem.domains[0].root_block_cm * problem.domains[0].nroot[0]
    qtot = sum(float(np.sum(q)) for q in problem.src_q)
    scale = qtot / (4.0 * np.pi * (0.25 * side) ** 2)
    f = scale * np.exp(sigma * rng.standard_normal(n))
    f[rng.random(n) < dark_fraction] = 0.0
    return f


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
