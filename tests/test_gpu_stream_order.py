"""Device index arrays (WR_DEVICE_INDEX) and stream order: two
wr_order_matrices calls and a wr_sssp call enqueued back to back on one
torch stream, with no synchronisation between them; each call's picks (or
sources) are written by torch kernels on that stream just before it, and
its outputs are device tensors.  Every result equals the oracle's."""
import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.gpu


def test_back_to_back_on_one_stream(rt):
    import torch
    ctx = rt.Context(0)
    wl = make_config("medium", side=96, num_orders=12)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 20)
    off, picks = wl.pick_offsets, wl.picks
    n = len(off) - 1
    total = int((np.diff(off.astype(np.int64)) ** 2).sum())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d_off = torch.from_numpy(off.view(np.int32).copy()).cuda()
        base = torch.from_numpy(picks.view(np.int32).copy()).cuda()
        p1 = base * 1                      # written by a kernel on the stream
        o1 = torch.empty(total, dtype=torch.int32, device="cuda")
        G.order_matrices(d_off, p1, out=o1)
        # the second batch: every order's picks reversed, written right after
        p2 = torch.cat([p1[int(off[o]):int(off[o + 1])].flip(0) for o in range(n)])
        o2 = torch.empty(total, dtype=torch.int32, device="cuda")
        G.order_matrices(d_off, p2, out=o2)
        src = p2[:5] + 0
        rows = torch.empty(5 * g.V, dtype=torch.int32, device="cuda")
        G.sssp(src, out=rows)
    s.synchronize()
    picks2 = np.concatenate([picks[off[o]:off[o + 1]][::-1] for o in range(n)]).astype(np.uint32)
    assert (o1.cpu().numpy().view(np.uint32) == oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)).all()
    assert (o2.cpu().numpy().view(np.uint32) == oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks2)).all()
    er = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, picks2[:5])
    assert (rows.cpu().numpy().view(np.uint32).reshape(5, g.V) == er).all()
    G.close()


def test_device_index_bad_input(rt):
    """A device pick out of range fails the call like a host one."""
    import torch
    ctx = rt.Context(0)
    wl = make_config("medium", side=48, num_orders=2)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    off = torch.from_numpy(wl.pick_offsets.view(np.int32).copy()).cuda()
    pk = torch.from_numpy(wl.picks.view(np.int32).copy()).cuda()
    pk[3] = g.V
    out = torch.empty(int((np.diff(wl.pick_offsets.astype(np.int64)) ** 2).sum()), dtype=torch.int32, device="cuda")
    with pytest.raises(rt.WrError) as e:
        G.order_matrices(off, pk, out=out)
    assert e.value.name == "WR_E_INVALID"
    G.close()
