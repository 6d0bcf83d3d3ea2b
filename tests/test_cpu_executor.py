"""The library's unchanged HIP kernels and host runtime, run on the CPU by the
test executor (tests/simt_cpu: lanes as threads, emulated wave collectives
and barriers, AddressSanitizer on every buffer), against the oracle.  This
checks the kernels' logic and bounds without a GPU; the GPU tests check the
same paths on the hardware."""
import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def harness():
    from tests.simt_cpu import harness as h
    h.driver(rebuild=True)
    return h


def test_overlay_order_matrices_tiny(harness):
    wl = make_config("tiny")
    g = wl.graph
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=wl.pick_offsets, picks=wl.picks,
                                  algo="overlay", seg=("grid", g.W, g.H, 1, g.W // 3, g.H // 3))
    assert st == 0, err[-2000:]
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (out == exp).all()


def test_segmented_rows_and_pred_random_graph(harness):
    from tests.helpers import random_csr
    rng = np.random.default_rng(31)
    V = 160
    rp, col, w = random_csr(rng, V, 4 * V, wmax=20)
    seg = rng.integers(0, 5, V).astype(np.uint32)
    src = rng.choice(V, 9, replace=False).astype(np.uint32)
    st, out, pred, err = harness.run(rp, col, w, sources=src, algo="segmented", pred=True,
                                     seg=("map", 5, seg))
    assert st == 0, err[-2000:]
    d = out.reshape(len(src), V)
    p = pred.reshape(len(src), V)
    for i, s in enumerate(src):
        ed = oracle.dijkstra(rp, col, w, int(s))
        assert (d[i] == ed).all()
        assert (p[i] == oracle.canonical_pred(rp, col, w, int(s), ed)).all()
