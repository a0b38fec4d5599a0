"""The C-ABI library loads and exports every entry point include/spv.h
declares (no GPU work: only symbol lookup)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spv.h")
LIB = os.path.join(ROOT, "paper_1702_02939_amd", "libspv.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spv_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("spv_create", "spv_step", "spv_get_positions", "spv_get_forces", "spv_get_neighbors",
                 "spv_destroy", "spv_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libspv.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_imports_and_uses_same_names():
    from paper_1702_02939_amd import spv
    for n in declared_functions():
        if n in ("spv_last_error",):
            continue
        assert hasattr(spv, n), n


def test_invalid_arguments_rejected_before_any_gpu_work():
    from paper_1702_02939_amd import spv
    import numpy as np
    with pytest.raises(spv.SPVError) as ei:
        spv.spv_create(2, np.zeros(2), np.zeros(2), 1.0, 1.0, params=spv.Params())
    assert ei.value.status == spv.SPV_EINVAL
    with pytest.raises(spv.SPVError) as ei:
        spv.spv_create(10, np.zeros(10), np.zeros(10), -1.0, 1.0, params=spv.Params())
    assert ei.value.status == spv.SPV_EINVAL
    with pytest.raises(spv.SPVError) as ei:
        spv.spv_create(10, np.zeros(10), np.zeros(10), 1.0, 1.0, params=spv.Params(kcap=100))
    assert ei.value.status == spv.SPV_EINVAL
    x = np.linspace(0.5, 9.5, 10)
    for kw in (dict(bin_factor=0.25), dict(bin_factor=9.0), dict(autotune=3), dict(repair_cells=-1),
               dict(device_rounds=-2), dict(full_rounds=5), dict(tail_items=-1), dict(bin_order=2),
               dict(force_mode=3), dict(force_mode=-1)):
        with pytest.raises(spv.SPVError) as ei:
            spv.spv_create(10, x, x[::-1].copy(), 10.0, 10.0, params=spv.Params(**kw))
        assert ei.value.status == spv.SPV_EINVAL, kw


def test_ring_extent_limit_rejected_before_reading_inputs():
    """N * kcap must stay below 2^30 (ring rows use 32-bit byte offsets); a
    larger system is refused on the host before any input is read or any
    device memory allocated -- here with 4-entry arrays standing in for
    tens of millions of cells, so reading them would be out of bounds."""
    from paper_1702_02939_amd import spv
    import numpy as np
    tiny = np.zeros(4)
    for N, kcap in ((1 << 26, 16), (1 << 25, 32), ((1 << 26) + 5, 0), (1 << 29, 16)):
        with pytest.raises(spv.SPVError) as ei:
            spv.spv_create(N, tiny, tiny, 8192.0, 8192.0, params=spv.Params(kcap=kcap))
        assert ei.value.status == spv.SPV_EINVAL
        assert "2^30" in str(ei.value)
    # batches: the total over the systems counts
    with pytest.raises(spv.SPVError) as ei:
        spv.spv_batch_create([1 << 25, 1 << 25], [5793.0, 5793.0], tiny, tiny, [3.8, 3.8],
                             params=spv.Params(kcap=16))
    assert ei.value.status == spv.SPV_EINVAL and "2^30" in str(ei.value)
