"""Host-side checks of the HIP library: it is built for gfx950, loads, and
exports every entry point that include/treeray.h declares.  No device calls."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2105_09644_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    import paper_2105_09644_amd as T
    return T.load_library()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "treeray.h")).read()
    return sorted(set(re.findall(r"\b(tr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    import paper_2105_09644_amd as T
    assert declared_symbols() == sorted(T.SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_library_holds_gfx950_code():
    from paper_2105_09644_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", B.LIB], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2105_09644_amd as T
    from paper_2105_09644_amd import workloads as W
    with pytest.raises(RuntimeError):
        T.context_for(W.small_uniform(8))


def test_stale_library_is_refused(tmp_path, monkeypatch):
    """A library whose compiled-in source digest differs from the sources in the
    tree is refused by the binding (no silent use of an old build)."""
    import shutil

    import paper_2105_09644_amd as T
    from paper_2105_09644_amd import build as B
    if B.stale():
        B.build()
    assert not B.stale()
    assert B.library_digest() == B.source_digest()
    copy = str(tmp_path / "libtreeray.so")
    shutil.copy(B.LIB, copy)
    monkeypatch.setattr(T, "_lib", None)
    monkeypatch.setattr(B, "source_digest", lambda: "0123456789abcdef")
    assert B.stale(copy)
    with pytest.raises(ImportError, match="other sources"):
        T.load_library(copy)
