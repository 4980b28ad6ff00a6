"""The C ABI library loads, exports every symbol include/burn.h declares, and
rejects bad calls on the host before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "burn.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2312_02836_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libburn.so not built")
    return _lib.lib()


def test_header_declares_expected(L):
    from paper_2312_02836_amd import _lib
    declared = _declared_functions()
    assert set(_lib.EXPORTS) == set(declared), declared


def test_every_declared_symbol_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_version_and_last_error(L):
    assert b"gfx950" in L.bn_version()
    assert isinstance(L.bn_last_error(), bytes)


def _desc(spec):
    from paper_2312_02836_amd import _lib
    arrs = [np.ascontiguousarray(spec.mass, dtype=np.int32),
            np.ascontiguousarray(spec.reactants, dtype=np.int32),
            np.ascontiguousarray(spec.products, dtype=np.int32),
            np.ascontiguousarray(spec.coef, dtype=np.float64),
            np.ascontiguousarray(spec.q, dtype=np.float64)]
    i32, f64 = C.POINTER(C.c_int32), C.POINTER(C.c_double)
    d = _lib.NetworkDesc(spec.n_species, spec.n_reactions, arrs[0].ctypes.data_as(i32),
                         arrs[1].ctypes.data_as(i32), arrs[2].ctypes.data_as(i32),
                         arrs[3].ctypes.data_as(f64), arrs[4].ctypes.data_as(f64), spec.c_v)
    return d, arrs


def test_network_validation_rejects_on_host(L):
    """Invalid descriptions are rejected before any device allocation."""
    from paper_2312_02836_amd import _lib, synth
    good = synth.robertson_network()
    h = C.c_void_p()
    # non-conserving reaction
    bad = synth.NetworkSpec.from_json(good.to_json())
    bad.mass[2] = 2
    d, keep = _desc(bad)
    assert L.bn_network_create(C.byref(d), C.byref(h)) == _lib.BN_EINVAL
    assert b"conserve" in L.bn_last_error()
    # index out of range
    bad = synth.NetworkSpec.from_json(good.to_json())
    bad.reactants[0, 0] = 7
    d, keep = _desc(bad)
    assert L.bn_network_create(C.byref(d), C.byref(h)) == _lib.BN_EINVAL
    # non-positive c_v
    bad = synth.NetworkSpec.from_json(good.to_json())
    bad.c_v = 0.0
    d, keep = _desc(bad)
    assert L.bn_network_create(C.byref(d), C.byref(h)) == _lib.BN_EINVAL
    # too large a system
    big = synth.chain_network([1.0] * 70)
    d, keep = _desc(big)
    assert L.bn_network_create(C.byref(d), C.byref(h)) == _lib.BN_EUNSUPPORTED
    # null arguments
    assert L.bn_network_create(None, C.byref(h)) == _lib.BN_EINVAL


def test_burn_rejects_bad_arguments_on_host(L):
    from paper_2312_02836_amd import _lib
    dummy = C.c_void_p(1)
    # null network
    assert L.burn_batch(None, 4, dummy, dummy, dummy, 1.0, 1e-6, 1e-10, None, None, None,
                        None) == _lib.BN_EINVAL
    L.bn_network_destroy(None)  # no-op
    assert L.bn_network_n_species(None) == -1


def test_multi_and_tuning_reject_bad_arguments_on_host(L):
    """Argument checks of the persistent and tuning entry points that come
    before any device call."""
    from paper_2312_02836_amd import _lib
    opts = _lib.BurnOpts(0, 0, 0, 0)
    items = (_lib.BatchItem * 1)()
    assert L.burn_batch_multi(-1, items, 1e-2, 1e-6, 1e-10, None, None, 0, None) == _lib.BN_EINVAL
    assert L.burn_batch_multi(9, items, 1e-2, 1e-6, 1e-10, None, None, 0, None) == _lib.BN_EINVAL
    assert L.burn_batch_multi(1, None, 1e-2, 1e-6, 1e-10, None, None, 0, None) == _lib.BN_EINVAL
    assert L.burn_batch_multi(1, items, 0.0, 1e-6, 1e-10, None, None, 0, None) == _lib.BN_EINVAL
    assert L.burn_batch_multi(1, items, 1e-2, 1e-6, -1.0, None, None, 0, None) == _lib.BN_EINVAL
    bad = _lib.BurnOpts(0, 4, 0, 0)
    assert L.burn_batch_multi(1, items, 1e-2, 1e-6, 1e-10, C.byref(bad), None, 0,
                              None) == _lib.BN_EINVAL
    assert b"lanes_per_cell" in L.bn_last_error()
    assert L.burn_batch_multi(0, items, 1e-2, 1e-6, 1e-10, C.byref(opts), None, 0,
                              None) in (_lib.BN_SUCCESS, _lib.BN_EHIP)
    assert L.burn_batch_multi_workspace_bytes(1) == 256
    assert L.burn_batch_multi_workspace_bytes(8) == 256
    # ordered queue: per item with cells 1 KiB of bucket counters, 8 queue
    # counters (one per XCD), h0 and the position (4 + 4 bytes per cell), staged state (8 N), T, rho (8 + 8),
    # status (4) and counters (32 bytes per cell), each region 256-byte
    # aligned; an item without a network counts N = 0
    two = (_lib.BatchItem * 2)()
    two[0].n_cells, two[1].n_cells = 1000, 0
    assert L.burn_batch_multi_order_workspace_bytes(2, None) == 256
    assert L.burn_batch_multi_order_workspace_bytes(2, two) == (
        256 + 1024 + 256 + 4096 + 4096 + 0 + 8192 + 8192 + 4096 + 32000)
    order_bad = _lib.BurnOpts(0, 0, 0, 2)
    assert L.burn_batch_multi(1, items, 1e-2, 1e-6, 1e-10, C.byref(order_bad), None, 0,
                              None) == _lib.BN_EINVAL
    assert b"order_cells" in L.bn_last_error()
    n = C.c_int32(5)
    assert L.bn_network_autotune(None, 10, None, None, None, 1e-2, 1e-6, 1e-10, None, 0, None,
                                 0, C.byref(n), None) == _lib.BN_EINVAL
    assert n.value == 0
    assert L.bn_network_set_launch(None, 4, 4, 0) == _lib.BN_EINVAL
    a = C.c_int32()
    assert L.bn_network_get_launch(None, C.byref(a), C.byref(a), C.byref(a)) == _lib.BN_EINVAL
