"""wr_order_routes_static (exact routes with no device allocation by the
library) against wr_order_routes on the same device inputs: two calls in a
row on one GPU, the second smaller, so what the first call left in the
library's fixed work array must not leak into the second."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _batch(rng, sizes):
    mats = []
    for n in sizes:
        D = rng.integers(1, 60, (n, n)).astype(np.uint32)   # small values: many ties
        np.fill_diagonal(D, 0)
        if n > 2:
            D[rng.integers(0, n), rng.integers(0, n)] = 0xFFFFFFFF
        mats.append(D.ravel())
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    flat = np.concatenate(mats).astype(np.uint32) if mats else np.zeros(0, np.uint32)
    return off, flat


@pytest.mark.parametrize("enum", [False, True], ids=["held_karp", "enumerate"])
def test_static_routes_equal_allocating_entry(rt, enum):
    import torch
    ctx = rt.Context(0)
    rng = np.random.default_rng(11 + enum)
    nmax = 8 if enum else 12
    for count in (700, 37):
        sizes = rng.integers(0, nmax + 1, count)
        off, flat = _batch(rng, sizes)
        print(f"static routes: enumerate={enum} orders={count} picks={int(off[-1])}", flush=True)
        exp_len, exp_rt = ctx.order_routes(off, flat, enumerate=enum)
        d = torch.from_numpy(flat.view(np.int32).copy()).cuda()
        ln = torch.full((count,), -1, dtype=torch.int64, device="cuda")
        rr = torch.full((max(int(off[-1]), 1),), -1, dtype=torch.int32, device="cuda")
        ctx.order_routes_static(off, d, ln, rr, enumerate=enum)
        torch.cuda.synchronize()
        assert (ln.cpu().numpy().view(np.uint64) == exp_len).all()
        assert (rr.cpu().numpy()[:int(off[-1])].view(np.uint32) == exp_rt).all()
    ctx.close()


def test_static_routes_reject_oversized_batches(rt):
    import torch
    ctx = rt.Context(0)
    n = 65537
    off = np.zeros(n + 1, np.uint32)
    d = torch.zeros(1, dtype=torch.int32, device="cuda")
    ln = torch.zeros(n, dtype=torch.int64, device="cuda")
    rr = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes_static(off, d, ln, rr)
    assert e.value.name == "WR_E_RANGE"
    # at the maximum the call runs (every order empty: lengths 0)
    ctx.order_routes_static(off[:65537], d, ln[:65536], rr)
    torch.cuda.synchronize()
    assert (ln[:65536].cpu().numpy() == 0).all()
    ctx.close()
