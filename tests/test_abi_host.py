"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/wroute.h declares, and validation statuses follow the
documented rules."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wroute.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(wr_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2504_20655_amd as wr
    L = wr.lib()
    names = _declared()
    assert "wr_sssp" in names and "wr_order_matrices" in names
    missing = [n for n in names if getattr(L, n, None) is None]
    assert not missing, missing
    assert set(names) == set(wr._lib.SIGNATURES)


def test_status_strings():
    import paper_2504_20655_amd as wr
    L = wr.lib()
    for code, name in wr.STATUS.items():
        assert L.wr_status_str(code).decode() == name


def test_validate_csr_statuses():
    import paper_2504_20655_amd as wr
    rp = np.asarray([0, 1, 2], np.uint32)
    col = np.asarray([1, 0], np.uint32)
    w = np.asarray([5, 5], np.uint32)
    assert wr.validate_csr(rp, col, w) == 0
    assert wr.validate_csr(np.asarray([0, 1, 3], np.uint32), col, w) == 1
    assert wr.validate_csr(np.asarray([0, 2, 1], np.uint32), col, w) == 1
    assert wr.validate_csr(np.asarray([1, 1, 2], np.uint32), col, w) == 1
    assert wr.validate_csr(rp, np.asarray([1, 2], np.uint32), w) == 1
    assert wr.validate_csr(rp, col, np.asarray([0xFFFFFFFF, 1], np.uint32)) == 2
    rp3 = np.asarray([0, 1, 2, 2, 2], np.uint32)
    col3 = np.asarray([1, 2], np.uint32)
    assert wr.validate_csr(rp3, col3, np.asarray([0x80000000, 1], np.uint32)) == 2
    assert wr.validate_csr(rp3, col3, np.asarray([0x7FFFFFFF, 1], np.uint32)) == 0
    L = wr.lib()
    assert L.wr_validate_csr(0, 0, None, None, None) == 1
    assert b"NULL" in L.wr_last_error() or L.wr_last_error() != b""


def test_validation_agrees_with_oracle_on_random_inputs():
    import oracle
    import paper_2504_20655_amd as wr
    rng = np.random.default_rng(0)
    for _ in range(200):
        V = int(rng.integers(1, 8))
        E = int(rng.integers(0, 10))
        rp = np.sort(rng.integers(0, E + 1, V + 1)).astype(np.uint32)
        rp[0] = 0
        if rng.random() < 0.7:
            rp[-1] = E
        if rng.random() < 0.2 and V > 1:
            rp[1], rp[0] = rp[0] + 1, rp[1]
        col = rng.integers(0, V + (1 if rng.random() < 0.2 else 0), E).astype(np.uint32)
        w = rng.integers(0, 2**32 if rng.random() < 0.2 else 100, E, dtype=np.uint64).astype(np.uint32)
        assert wr.validate_csr(rp, col, w) == oracle.validate_csr(rp, col, w)


def test_context_without_gpu_reports_device_error():
    import paper_2504_20655_amd as wr
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    with pytest.raises(wr.WrError) as ei:
        wr.Context(0)
    assert ei.value.name == "WR_E_DEVICE"


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2504_20655_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
