"""Builds ``libtreeray.so`` for gfx950 with hipcc (in-tree).

The library carries the digest of the sources it was built from
(``tr_source_digest``); :func:`stale` compares it with the digest of the
sources in the tree, so a library left over from older sources is refused
by the binding instead of being used.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtreeray.so")
SOURCES = ["treeray.hip", "topology.cpp"]
HEADERS = ["kernels.h", "tr_internal.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TREERAY_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def source_files():
    return ([os.path.join(CSRC, s) for s in SOURCES + HEADERS]
            + [os.path.join(ROOT, "include", "treeray.h"), os.path.abspath(__file__)])


def source_digest() -> str:
    """First 16 hex digits of the SHA-256 over the library's sources and this build script."""
    h = hashlib.sha256()
    for f in source_files():
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def library_digest(path: str = LIB):
    """The source digest compiled into the library at path (None if it has none)."""
    try:
        L = ctypes.CDLL(path)
        f = L.tr_source_digest
    except (OSError, AttributeError):
        return None
    f.restype = ctypes.c_char_p
    f.argtypes = []
    v = f()
    return v.decode() if v else None


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, f'-DTR_SOURCE_DIGEST="{source_digest()}"', "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libtreeray.so")
    # the host pass warns about the device-only feature flag; anything else is shown
    noise = [ln for ln in (res.stdout + res.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "warning generated" not in ln]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")
    os.replace(tmp, LIB)
    return LIB


def stale(path: str = LIB) -> bool:
    """True when the library at path is missing or was built from other sources."""
    if not os.path.exists(path):
        return True
    return library_digest(path) != source_digest()


if __name__ == "__main__":
    print(build(verbose=True))
