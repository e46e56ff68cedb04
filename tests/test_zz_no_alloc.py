"""tr_delta_noalloc (through the C ABI): delta_cell per domain with no context
and no allocation, against tr_delta of a context on the same cells and against
the oracle's delta_cell; two calls in a row on one device (the second with a
smaller input, so that it reuses the static scratch the first one left)."""
import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import paper_2105_09644_amd as T
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    T.load_library()
    return T


def fields(T, P):
    """An optically thin sweep and the absorbing sweep after it (FP64)."""
    ctx = T.context_for(P, T.TR_FP64)
    nh = torch.tensor(np.concatenate(P.n_h), dtype=torch.float64, device="cuda")
    f0 = torch.zeros(ctx.n_cells, dtype=torch.float64, device="cuda")
    f1 = torch.zeros_like(f0)
    ctx.build(nh, None, thin=True)
    ctx.sweep(f0)
    ctx.build(nh, f0)
    ctx.sweep(f1)
    ctx.sync()
    return ctx, f0, f1


def test_delta_without_allocation_matches_tr_delta(T, orc):
    P = W.config4(n_domains=5, sizes=(16, 24, 32))
    ctx, f_old, f_new = fields(T, P)
    counts = [d.n_cells() for d in P.domains]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ref = ctx.delta(f_new, f_old)
    ctx.close()
    out = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    T.delta_noalloc(f_new, f_old, off, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    print("noalloc", got, "tr_delta", ref, flush=True)
    assert np.array_equal(got, ref)
    fo, fn = f_old.cpu().numpy(), f_new.cpu().numpy()
    for d in range(5):
        assert got[d] == pytest.approx(orc.delta_cell(fn[off[d]:off[d + 1]], fo[off[d]:off[d + 1]]), rel=1e-15)

    # second call, smaller input (two domains): the scratch keeps the first
    # call's state, which the call must not read
    P2 = W.Problem(P.name, P.domains[:2], P.n_h[:2], P.src_xyz[:2], P.src_q[:2], P.params)
    ctx2, g_old, g_new = fields(T, P2)
    ref2 = ctx2.delta(g_new, g_old)
    ctx2.close()
    out2 = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    T.delta_noalloc(g_new, g_old, off[:3], out2)
    torch.cuda.synchronize()
    got2 = out2.cpu().numpy()
    print("noalloc", got2, "tr_delta", ref2, flush=True)
    assert np.array_equal(got2, ref2)

    # beyond the scratch's 64 domains, and bad offsets: refused with a message
    big = np.arange(66, dtype=np.int64)
    with pytest.raises(T.TreeRayError, match="64"):
        T.delta_noalloc(f_new, f_old, big, torch.zeros(65, dtype=torch.float64, device="cuda"))
    with pytest.raises(T.TreeRayError, match="strictly increasing"):
        T.delta_noalloc(f_new, f_old, np.array([0, 5, 5], np.int64), out2)
