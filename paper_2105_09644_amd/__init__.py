"""TreeRay/OnTheSpot on MI355X: Python binding of ``libtreeray.so``.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device memory and streams come from PyTorch (ROCm); the binding
passes raw pointers across the C ABI declared in ``include/treeray.h``.
There is no fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtreeray.so")

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EHIP, TR_ENOCONV, TR_ESTATE, TR_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
TR_FP64, TR_FP32C = 0, 1

# every entry point of include/treeray.h
SYMBOLS = ["tr_create", "tr_set_domains", "tr_cell_count", "tr_set_sources", "tr_build", "tr_sweep",
           "tr_sweep_targets", "tr_delta", "tr_step", "tr_solve", "tr_set_precision", "tr_set_launch", "tr_autotune",
           "tr_get_stats", "tr_sync", "tr_last_error", "tr_destroy", "tr_source_digest", "tr_delta_noalloc"]


class TreeRayError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"treeray status {status}: {msg}")
        self.status = status


class _Domain(C.Structure):
    _fields_ = [("nroot", C.c_int32 * 3), ("max_level", C.c_int32), ("root_block_cm", C.c_double),
                ("n_leaf_blocks", C.c_int64), ("leaf_blocks", C.POINTER(C.c_int32))]


class _Params(C.Structure):
    _fields_ = [("nside", C.c_int32), ("n_radial", C.c_int32), ("eta_r", C.c_double), ("theta", C.c_double),
                ("alpha_b", C.c_double), ("hnu_erg", C.c_double), ("eps_lim", C.c_double),
                ("subsample", C.c_int32), ("max_iter", C.c_int32), ("zeta_g", C.c_int32), ("precision", C.c_int32),
                ("theta_if", C.c_double), ("theta_src", C.c_double), ("src_radius_cm", C.c_double),
                ("eps_kernel", C.c_int32), ("mass_kernel", C.c_int32), ("periodic", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_nodes", C.c_int64), ("nodes_accepted", C.c_int64),
                ("nodes_tested", C.c_int64), ("guard_recomputes", C.c_int64), ("n_radial_max", C.c_int32),
                ("depth_max", C.c_int32), ("waves_per_target", C.c_int32), ("targets_per_cu", C.c_int32),
                ("buffer_in_lds", C.c_int32), ("overflow", C.c_int32), ("integration_wave", C.c_int32),
                ("lds_cas", C.c_int32), ("integration_fp32", C.c_int32),
                ("last_sweep_ms", C.c_double), ("rays_fp32", C.c_int64), ("rays_fp64_again", C.c_int64),
                ("nodes_tabulated", C.c_int64), ("rays_regrouped", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the HIP library; raises if it is missing or was built from other
    sources than those in the tree (there is no CPU path and no silent use of
    a stale build)."""
    global _lib
    if _lib is not None:
        return _lib
    from . import build as _build
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or "
                          f"python -m paper_2105_09644_amd.build")
    if _build.stale(path):
        raise ImportError(f"{path} was built from other sources (digest {_build.library_digest(path)}, "
                          f"sources {_build.source_digest()}); rebuild it with __graft_entry__.build()")
    L = C.CDLL(path)
    vp, dp, i64p, u8p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_uint8)
    sig = {
        "tr_create": ([C.POINTER(vp), C.POINTER(_Params), vp], C.c_int),
        "tr_set_domains": ([vp, C.c_int32, C.POINTER(_Domain)], C.c_int),
        "tr_cell_count": ([vp, C.c_int32, i64p], C.c_int),
        "tr_set_sources": ([vp, C.c_int32, C.c_int64, dp, dp], C.c_int),
        "tr_build": ([vp, vp, vp, C.c_int32], C.c_int),
        "tr_sweep": ([vp, vp, vp], C.c_int),
        "tr_sweep_targets": ([vp, vp, C.c_int64, vp, vp], C.c_int),
        "tr_delta": ([vp, vp, vp, dp], C.c_int),
        "tr_step": ([vp, vp, vp, vp, vp, dp], C.c_int),
        "tr_solve": ([vp, vp, vp, vp, C.POINTER(C.c_int32), dp], C.c_int),
        "tr_set_precision": ([vp, C.c_int32], C.c_int),
        "tr_set_launch": ([vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32], C.c_int),
        "tr_autotune": ([vp, dp], C.c_int),
        "tr_get_stats": ([vp, C.POINTER(Stats)], C.c_int),
        "tr_sync": ([vp], C.c_int),
        "tr_last_error": ([vp], C.c_char_p),
        "tr_destroy": ([vp], None),
        "tr_source_digest": ([], C.c_char_p),
        "tr_delta_noalloc": ([vp, vp, i64p, C.c_int32, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def delta_noalloc(f_new, f_old, dom_offsets, delta_out, stream=None):
    """tr_delta_noalloc: delta_cell per domain into the device tensor delta_out
    (float64 [n_domains]) without a context or an allocation; dom_offsets are
    the n_domains + 1 cell offsets (host)."""
    import torch
    L = load_library()
    off = np.ascontiguousarray(dom_offsets, dtype=np.int64)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = L.tr_delta_noalloc(_ptr(f_new), _ptr(f_old), off.ctypes.data_as(C.POINTER(C.c_int64)), len(off) - 1,
                            _ptr(delta_out), C.c_void_p(st.cuda_stream))
    if rc != TR_OK:
        msg = L.tr_last_error(None)
        raise TreeRayError(rc, msg.decode() if msg else "")


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """One library context on the current GPU and torch's current stream.

    ``domains`` are :class:`paper_2105_09644_amd.workloads.Domain` objects; the
    cell arrays passed to :meth:`build`, :meth:`sweep` and :meth:`solve` are
    torch tensors on the GPU (float64 densities and fluxes, uint8 flags).
    """

    def __init__(self, params, domains, precision=TR_FP64, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("treeray needs a GPU: torch.cuda.is_available() is False")
        self.torch = torch
        self.L = load_library()
        p = _Params()
        p.nside = int(params.nside)
        p.n_radial = int(params.n_radial)
        p.eta_r = float(params.eta_r)
        p.theta = float(params.theta)
        p.alpha_b = float(params.alpha_b)
        p.hnu_erg = 13.6 * 1.602176634e-12
        p.eps_lim = float(params.eps_lim)
        p.subsample = int(params.subsample)
        p.max_iter = int(params.max_iter)
        p.zeta_g = int(bool(params.zeta_g))
        p.precision = int(precision)
        p.theta_if = float(getattr(params, "theta_if", 0.0))
        p.theta_src = float(getattr(params, "theta_src", 0.0))
        p.src_radius_cm = float(getattr(params, "src_radius_cm", 0.0))
        p.eps_kernel = int(getattr(params, "eps_kernel", 0))
        p.mass_kernel = int(getattr(params, "mass_kernel", 0))
        p.periodic = int(bool(getattr(params, "periodic", False)))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(self.L.tr_create(C.byref(h), C.byref(p), C.c_void_p(self.stream.cuda_stream)), None)
        self.h = h
        self._keep = []
        arr = (_Domain * len(domains))()
        for i, d in enumerate(domains):
            for a in range(3):
                arr[i].nroot[a] = int(d.nroot[a])
            arr[i].max_level = int(d.max_level)
            arr[i].root_block_cm = float(d.root_block_cm)
            if d.leaf_blocks is None:
                arr[i].n_leaf_blocks = 0
                arr[i].leaf_blocks = None
            else:
                lb = np.ascontiguousarray(d.leaf_blocks, dtype=np.int32)
                self._keep.append(lb)
                arr[i].n_leaf_blocks = lb.shape[0]
                arr[i].leaf_blocks = lb.ctypes.data_as(C.POINTER(C.c_int32))
        self._check(self.L.tr_set_domains(self.h, len(domains), arr))
        self.n_domains = len(domains)
        n = C.c_int64()
        self._check(self.L.tr_cell_count(self.h, -1, C.byref(n)))
        self.n_cells = n.value

    def _check(self, rc, h="self"):
        if rc != TR_OK:
            msg = self.L.tr_last_error(self.h if h == "self" else None)
            raise TreeRayError(rc, msg.decode() if msg else "")
        return rc

    def cell_count(self, dom=-1):
        n = C.c_int64()
        self._check(self.L.tr_cell_count(self.h, int(dom), C.byref(n)))
        return n.value

    def set_sources(self, dom, xyz_cm, q):
        xyz = np.ascontiguousarray(xyz_cm, dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).ravel()
        self._check(self.L.tr_set_sources(self.h, int(dom), len(q), xyz.ctypes.data_as(C.POINTER(C.c_double)),
                                          q.ctypes.data_as(C.POINTER(C.c_double))))

    def set_precision(self, prec):
        self._check(self.L.tr_set_precision(self.h, int(prec)))

    def set_launch(self, waves=0, targets_per_cu=0, buffer=0, integration=0, atomics=0):
        self._check(self.L.tr_set_launch(self.h, int(waves), int(targets_per_cu), int(buffer), int(integration),
                                         int(atomics)))

    def autotune(self):
        ms = C.c_double()
        self._check(self.L.tr_autotune(self.h, C.byref(ms)))
        return ms.value

    def build(self, n_h, f_prev=None, thin=False):
        self._check(self.L.tr_build(self.h, _ptr(n_h), _ptr(f_prev), int(bool(thin))))

    def sweep(self, f_out, ion_out=None):
        self._check(self.L.tr_sweep(self.h, _ptr(f_out), _ptr(ion_out)))

    def sweep_targets(self, targets, f_out, ion_out=None):
        self._check(self.L.tr_sweep_targets(self.h, _ptr(targets), int(targets.numel()), _ptr(f_out),
                                            _ptr(ion_out)))

    def delta(self, f_new, f_old):
        out = np.zeros(self.n_domains)
        self._check(self.L.tr_delta(self.h, _ptr(f_new), _ptr(f_old), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def step(self, n_h, f_prev, f_out, ion_out=None):
        """One outer iteration (build, sweep, delta_cell) as a captured hipGraph."""
        out = np.zeros(self.n_domains)
        self._check(self.L.tr_step(self.h, _ptr(n_h), _ptr(f_prev), _ptr(f_out), _ptr(ion_out),
                                   out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def solve(self, n_h, f_out, ion_out=None, allow_noconv=False):
        it = C.c_int32()
        dl = C.c_double()
        rc = self.L.tr_solve(self.h, _ptr(n_h), _ptr(f_out), _ptr(ion_out), C.byref(it), C.byref(dl))
        if not (rc == TR_OK or (allow_noconv and rc == TR_ENOCONV)):
            self._check(rc)
        return it.value, dl.value

    def stats(self):
        s = Stats()
        self._check(self.L.tr_get_stats(self.h, C.byref(s)))
        return s

    def sync(self):
        self._check(self.L.tr_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.tr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def context_for(problem, precision=TR_FP64, **param_over):
    """Context with the problem's domains and sources declared."""
    import copy
    p = copy.copy(problem.params)
    for k, v in param_over.items():
        setattr(p, k, v)
    ctx = Context(p, problem.domains, precision=precision)
    for d in range(len(problem.domains)):
        ctx.set_sources(d, problem.src_xyz[d], problem.src_q[d])
    return ctx
