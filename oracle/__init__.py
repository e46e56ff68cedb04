"""FP64 CPU oracle for the TreeRay/OnTheSpot sweep -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``treeray_oracle.c`` (plain C,
FP64, OpenMP over target cells) with ctypes.  It shares no code with the HIP
library and never calls it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "treeray_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Domain(C.Structure):
    _fields_ = [("nroot", C.c_int32 * 3), ("max_level", C.c_int32), ("root_block_cm", C.c_double),
                ("n_leaf_blocks", C.c_int64), ("leaf_blocks", C.POINTER(C.c_int32))]


class Params(C.Structure):
    _fields_ = [("nside", C.c_int32), ("n_radial", C.c_int32), ("eta_r", C.c_double),
                ("theta", C.c_double), ("alpha_b", C.c_double), ("subsample", C.c_int32),
                ("zeta_g", C.c_int32), ("theta_if", C.c_double), ("theta_src", C.c_double),
                ("src_radius_cm", C.c_double), ("eps_kernel", C.c_int32), ("mass_kernel", C.c_int32),
                ("periodic", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("nodes_accepted", C.c_int64), ("nodes_tested", C.c_int64),
                ("n_nodes", C.c_int64), ("n_radial", C.c_int32), ("depth", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        u8p = C.POINTER(C.c_uint8)
        L.orc_cell_count.restype = C.c_int64
        L.orc_cell_count.argtypes = [C.POINTER(Domain)]
        L.orc_cell_geometry.argtypes = [C.POINTER(Domain), i64p, i64p]
        L.orc_radial_points.argtypes = [C.POINTER(Domain), C.POINTER(Params), C.c_int32, dp]
        L.orc_sweep.argtypes = [C.POINTER(Domain), C.POINTER(Params), dp, C.c_int64, dp, dp, dp,
                                C.c_int64, i64p, dp, u8p, C.POINTER(Stats)]
        L.orc_sweep_timed.argtypes = [C.POINTER(Domain), C.POINTER(Params), dp, C.c_int64, dp, dp, dp,
                                      C.c_int64, i64p, dp, u8p, C.POINTER(Stats), C.c_int32, dp]
        L.orc_node_pixels.restype = C.c_int32
        L.orc_node_pixels.argtypes = [C.c_int32, C.c_int32, i64p, i64p, dp, i64p, C.POINTER(C.c_int32)]
        L.orc_target_rays.restype = C.c_int32
        L.orc_target_rays.argtypes = [C.POINTER(Domain), C.POINTER(Params), dp, C.c_int64, dp, dp, dp, C.c_int64,
                                      C.c_int32, dp, dp, dp, dp]
        L.orc_solve.argtypes = [C.POINTER(Domain), C.POINTER(Params), dp, C.c_int64, dp, dp,
                                C.c_double, C.c_int32, dp, u8p, C.POINTER(C.c_int32), dp]
        L.orc_deposit.argtypes = [C.POINTER(Domain), C.c_int64, dp, dp, dp]
        L.orc_deposit_spheres.argtypes = [C.POINTER(Domain), C.c_int64, dp, dp, C.c_double, dp]
        L.orc_ball_box_volume.restype = C.c_double
        L.orc_wg.restype = C.c_double
        L.orc_wg.argtypes = [C.c_double]
        L.orc_mass_weights.argtypes = [C.c_int32, C.c_int32, dp, C.c_double, C.c_double, dp]
        L.orc_eps_weights.argtypes = [C.c_int32, C.c_int32, dp, C.c_double, C.c_double, dp]
        L.orc_ball_box_volume.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_delta_cell.restype = C.c_double
        L.orc_delta_cell.argtypes = [C.c_int64, dp, dp]
        L.orc_delta_tot.restype = C.c_double
        L.orc_delta_tot.argtypes = [C.c_int64, dp, dp, dp]
        L.orc_ang2pix.restype = C.c_int64
        L.orc_ang2pix.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_pix2vec.argtypes = [C.c_int32, C.c_int64, dp]
        L.orc_ang2pix_many.argtypes = [C.c_int32, C.c_int64, dp, i64p]
        L.orc_num_threads.restype = C.c_int32
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [C.c_int32]
        L.orc_wp.restype = C.c_double
        L.orc_wp.argtypes = [C.c_double]
        L.orc_wp_weights.argtypes = [C.c_int32, dp, C.c_double, C.c_double, dp]
        L.orc_wf3_weights.argtypes = [C.c_int32, dp, C.c_double, dp]
        L.orc_integrate_ray.restype = C.c_double
        L.orc_integrate_ray.argtypes = [C.c_int32, dp, dp, dp, dp, dp, C.c_int32, C.c_int32]
        L.orc_accepted.restype = C.c_int64
        L.orc_accepted.argtypes = [C.POINTER(Domain), C.POINTER(Params), dp, C.c_int64, dp, dp, dp,
                                   C.c_int64, C.c_int64, i64p, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _c_domain(dom):
    d = Domain()
    for a in range(3):
        d.nroot[a] = int(dom.nroot[a])
    d.max_level = int(dom.max_level)
    d.root_block_cm = float(dom.root_block_cm)
    if dom.leaf_blocks is None:
        d.n_leaf_blocks = 0
        d.leaf_blocks = None
        keep = None
    else:
        keep = np.ascontiguousarray(dom.leaf_blocks, dtype=np.int32)
        d.n_leaf_blocks = keep.shape[0]
        d.leaf_blocks = keep.ctypes.data_as(C.POINTER(C.c_int32))
    return d, keep


def _c_params(p, **over):
    q = Params()
    q.nside = int(over.get("nside", p.nside))
    q.n_radial = int(over.get("n_radial", p.n_radial))
    q.eta_r = float(over.get("eta_r", p.eta_r))
    q.theta = float(over.get("theta", p.theta))
    q.alpha_b = float(over.get("alpha_b", p.alpha_b))
    q.subsample = int(over.get("subsample", p.subsample))
    q.zeta_g = int(bool(over.get("zeta_g", p.zeta_g)))
    q.theta_if = float(over.get("theta_if", getattr(p, "theta_if", 0.0)))
    q.theta_src = float(over.get("theta_src", getattr(p, "theta_src", 0.0)))
    q.src_radius_cm = float(over.get("src_radius_cm", getattr(p, "src_radius_cm", 0.0)))
    q.eps_kernel = int(over.get("eps_kernel", getattr(p, "eps_kernel", 0)))
    q.mass_kernel = int(over.get("mass_kernel", getattr(p, "mass_kernel", 0)))
    q.periodic = int(bool(over.get("periodic", getattr(p, "periodic", False))))
    return q


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def cell_count(dom) -> int:
    d, keep = _c_domain(dom)
    return int(lib().orc_cell_count(C.byref(d)))


def cell_geometry(dom):
    n = cell_count(dom)
    d, keep = _c_domain(dom)
    lo = np.zeros((n, 3), np.int64)
    sz = np.zeros(n, np.int64)
    _check(lib().orc_cell_geometry(C.byref(d), lo.ctypes.data_as(C.POINTER(C.c_int64)),
                                   sz.ctypes.data_as(C.POINTER(C.c_int64))), "cell_geometry")
    return lo, sz


def radial_points(dom, params, **over):
    d, keep = _c_domain(dom)
    p = _c_params(params, **over)
    r = np.zeros(1024)
    n = lib().orc_radial_points(C.byref(d), C.byref(p), 1024, _dp(r))
    _check(n, "radial_points")
    return r[:n].copy()


def deposit(dom, xyz, q, radius_cm=0.0):
    """Source rates per cell; radius_cm > 0: sources are uniform spheres."""
    n = cell_count(dom)
    d, keep = _c_domain(dom)
    out = np.zeros(n)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    if radius_cm > 0:
        _check(lib().orc_deposit_spheres(C.byref(d), len(q), _dp(xyz), _dp(q), float(radius_cm), _dp(out)),
               "deposit")
    else:
        _check(lib().orc_deposit(C.byref(d), len(q), _dp(xyz), _dp(q), _dp(out)), "deposit")
    return out


K_DEFAULT, K_F1, K_F2, K_F3, K_F3N, K_P, K_G = 0, 1, 2, 3, 4, 5, 6


def wg(x):
    return float(lib().orc_wg(float(x)))


def mass_weights(kind, r, d, h):
    r = np.ascontiguousarray(r, dtype=np.float64)
    v = np.zeros(len(r))
    lib().orc_mass_weights(int(kind), len(r), _dp(r), float(d), float(h), _dp(v))
    return v


def eps_weights(kind, r, d, h):
    r = np.ascontiguousarray(r, dtype=np.float64)
    u = np.zeros(len(r))
    lib().orc_eps_weights(int(kind), len(r), _dp(r), float(d), float(h), _dp(u))
    return u


def ball_box_volume(centre, radius, lo, hi):
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    return float(lib().orc_ball_box_volume(float(centre[0]), float(centre[1]), float(centre[2]), float(radius),
                                           _dp(lo), _dp(hi)))


def sweep(dom, params, n_h, xyz, q, f_prev=None, targets=None, threads=0, timing=None, **over):
    """One sweep; returns (F_tot per target, ionised flag per target, stats).
    threads > 0 runs the target loop on that many threads; a list passed as
    timing receives the loop's wall time in seconds (tree build excluded)."""
    n = cell_count(dom)
    d, keep = _c_domain(dom)
    p = _c_params(params, **over)
    n_h = np.ascontiguousarray(n_h, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    fp = None if f_prev is None else np.ascontiguousarray(f_prev, dtype=np.float64)
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = len(targets), targets.ctypes.data_as(C.POINTER(C.c_int64))
    f = np.zeros(nt)
    ion = np.zeros(nt, np.uint8)
    st = Stats()
    sec = C.c_double(0.0)
    _check(lib().orc_sweep_timed(C.byref(d), C.byref(p), _dp(n_h), len(q), _dp(xyz), _dp(q), _dp(fp),
                                 nt, tp, _dp(f), ion.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(st),
                                 int(threads), C.byref(sec)),
           "sweep")
    if timing is not None:
        timing.append(sec.value)
    return f, ion, st


def node_pixels(nside, s, olo, ohi, xt):
    """Angular weights of the node box [olo, ohi) (finest-cell units) seen from
    the point xt: {pixel: sub-point count} over its s^3 sub-box midpoints."""
    olo = np.ascontiguousarray(olo, dtype=np.int64)
    ohi = np.ascontiguousarray(ohi, dtype=np.int64)
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    pix = np.zeros(s ** 3, np.int64)
    cnt = np.zeros(s ** 3, np.int32)
    n = lib().orc_node_pixels(int(nside), int(s), olo.ctypes.data_as(C.POINTER(C.c_int64)),
                              ohi.ctypes.data_as(C.POINTER(C.c_int64)), _dp(xt),
                              pix.ctypes.data_as(C.POINTER(C.c_int64)), cnt.ctypes.data_as(C.POINTER(C.c_int32)))
    _check(n, "node_pixels")
    return {int(pix[k]): int(cnt[k]) for k in range(n)}


def target_rays(dom, params, n_h, xyz, q, target, f_prev=None, **over):
    """Mapped ray buffers of one target before the integration: (eps, A, E, V),
    each [N_PIX, N_R], cgs, the self term included."""
    d, keep = _c_domain(dom)
    p = _c_params(params, **over)
    n_h = np.ascontiguousarray(n_h, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    fp = None if f_prev is None else np.ascontiguousarray(f_prev, dtype=np.float64)
    npix = 12 * p.nside ** 2
    cap = 1024
    bufs = [np.zeros(npix * cap) for _ in range(4)]
    nr = lib().orc_target_rays(C.byref(d), C.byref(p), _dp(n_h), len(q), _dp(xyz), _dp(q), _dp(fp), int(target),
                               cap, *[_dp(b) for b in bufs])
    _check(nr, "target_rays")
    return tuple(b[:npix * nr].reshape(npix, nr).copy() for b in bufs)


def solve(dom, params, n_h, xyz, q, eps_lim=1e-2, max_iter=30, **over):
    n = cell_count(dom)
    d, keep = _c_domain(dom)
    p = _c_params(params, **over)
    n_h = np.ascontiguousarray(n_h, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.zeros(n)
    ion = np.zeros(n, np.uint8)
    it = C.c_int32(0)
    dl = C.c_double(0)
    _check(lib().orc_solve(C.byref(d), C.byref(p), _dp(n_h), len(q), _dp(xyz), _dp(q),
                           float(eps_lim), int(max_iter), _dp(f),
                           ion.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(it), C.byref(dl)),
           "solve")
    return f, ion, it.value, dl.value


def delta_cell(f_new, f_old):
    f_new = np.ascontiguousarray(f_new, dtype=np.float64)
    f_old = np.ascontiguousarray(f_old, dtype=np.float64)
    return lib().orc_delta_cell(len(f_new), _dp(f_new), _dp(f_old))


def delta_tot(f_new, f_old, dv):
    f_new = np.ascontiguousarray(f_new, dtype=np.float64)
    f_old = np.ascontiguousarray(f_old, dtype=np.float64)
    dv = np.ascontiguousarray(dv, dtype=np.float64)
    return lib().orc_delta_tot(len(f_new), _dp(f_new), _dp(f_old), _dp(dv))


def ang2pix(nside, v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 3))
    out = np.zeros(v.shape[0], np.int64)
    lib().orc_ang2pix_many(int(nside), v.shape[0], _dp(v), out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out


def pix2vec(nside, pix):
    out = np.zeros(3)
    lib().orc_pix2vec(nside, int(pix), _dp(out))
    return out


def wp(x):
    return lib().orc_wp(float(x))


def wp_weights(r, d, h):
    r = np.ascontiguousarray(r, dtype=np.float64)
    v = np.zeros_like(r)
    lib().orc_wp_weights(len(r), _dp(r), float(d), float(h), _dp(v))
    return v


def wf3_weights(r, d):
    r = np.ascontiguousarray(r, dtype=np.float64)
    u = np.zeros_like(r)
    lib().orc_wf3_weights(len(r), _dp(r), float(d), _dp(u))
    return u


def integrate_ray(r, eps, A, E, V, nside, zeta_g=True):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (r, eps, A, E, V)]
    return lib().orc_integrate_ray(len(arr[0]), *[_dp(x) for x in arr], int(nside), int(zeta_g))


def accepted(dom, params, n_h, xyz, q, target, f_prev=None, **over):
    """Accepted nodes of one target: (lo_size [m,4], moments [m,9] =
    eps, alpha, E, V, mass, com xyz, ionised mass)."""
    d, keep = _c_domain(dom)
    p = _c_params(params, **over)
    n_h = np.ascontiguousarray(n_h, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    fp = None if f_prev is None else np.ascontiguousarray(f_prev, dtype=np.float64)
    cap = 1 << 16
    while True:
        ls = np.zeros((cap, 4), np.int64)
        mom = np.zeros((cap, 9))
        n = lib().orc_accepted(C.byref(d), C.byref(p), _dp(n_h), len(q), _dp(xyz), _dp(q), _dp(fp),
                               int(target), cap, ls.ctypes.data_as(C.POINTER(C.c_int64)), _dp(mom))
        _check(n, "accepted")
        if n <= cap:
            return ls[:n].copy(), mom[:n].copy()
        cap = int(n)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle sweeps (OpenMP)."""
    lib().orc_set_num_threads(int(n))
