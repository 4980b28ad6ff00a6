"""burn_batch_multi_noalloc (the multi-network launch whose scratch is the
library's static device array) against burn_batch_multi with a caller
workspace: bitwise equal results on two calls in a row, the second with a
smaller input, ordered and unordered; a launch that needs more scratch than
the array holds is rejected without running."""
import ctypes as C

import numpy as np
import pytest

from paper_2312_02836_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2312_02836_amd import _lib
    from paper_2312_02836_amd import burn as B
    return B, _lib


def _items(B, _lib, nets, cell_sets, dev):
    """Device copies of the cells and the bn_batch_item array over them."""
    import torch
    keep, items = [], (_lib.BatchItem * len(nets))()
    for j, (net, cells) in enumerate(zip(nets, cell_sets)):
        C_ = cells.n_cells
        Y = torch.as_tensor(cells.Y, device=dev).contiguous().clone()
        T = torch.as_tensor(cells.T, device=dev).contiguous().clone()
        rho = torch.as_tensor(cells.rho, device=dev).contiguous()
        st = torch.full((C_,), -7, dtype=torch.int32, device=dev)
        cnt = torch.full((8, C_), -7, dtype=torch.int32, device=dev)
        keep.append((Y, T, rho, st, cnt))
        items[j] = _lib.BatchItem(net.handle.value, C_, Y.data_ptr(), rho.data_ptr(),
                                  T.data_ptr(), None, st.data_ptr(), cnt.data_ptr())
    return keep, items


def _run_both(B, _lib, nets, cell_sets, t_end, order):
    import torch
    dev = torch.device("cuda", 0)
    L = _lib.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    opts = _lib.BurnOpts(0, 0, 0, order)
    ref, items_r = _items(B, _lib, nets, cell_sets, dev)
    nb = (L.burn_batch_multi_order_workspace_bytes(len(nets), items_r) if order
          else L.burn_batch_multi_workspace_bytes(len(nets)))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _lib.check(L.burn_batch_multi(len(nets), items_r, t_end, 1e-6, 1e-10, C.byref(opts),
                                  C.c_void_p(ws.data_ptr()), nb, stream), "burn_batch_multi")
    got, items_g = _items(B, _lib, nets, cell_sets, dev)
    _lib.check(L.burn_batch_multi_noalloc(len(nets), items_g, t_end, 1e-6, 1e-10,
                                          C.byref(opts), stream), "burn_batch_multi_noalloc")
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        assert (b[3] == 0).all()  # every cell burned to t_end
    return got


@pytest.mark.parametrize("order", [1, 0])
def test_noalloc_equals_workspace_launch(gpu, order):
    B, _lib = gpu
    c2 = synth.config(2, n_cells=3000)
    c5 = synth.config(5, n_cells=1000)
    nets = [B.Network(c2.networks[0]), B.Network(c5.networks[0])]
    # first call: two networks; second call: one network, fewer cells (the
    # scratch keeps the first call's contents, which must not leak in)
    _run_both(B, _lib, nets, [c2.cells[0], c5.cells[0]], c2.t_end, order)
    _run_both(B, _lib, nets[:1], [c2.cells[0].subset(np.arange(517))], c2.t_end, order)
    for n in nets:
        n.close()


def test_noalloc_rejects_launches_beyond_the_scratch(gpu):
    import torch
    B, _lib = gpu
    L = _lib.lib()
    spec = synth.config(2, n_cells=4).networks[0]
    net = B.Network(spec)
    C_ = 500_000  # ordered: 8 (N + 8) bytes per cell, more than 64 MiB
    dev = torch.device("cuda", 0)
    Y = torch.full((spec.n_species, C_), 0.1, dtype=torch.float64, device=dev)
    T = torch.full((C_,), 2.0, dtype=torch.float64, device=dev)
    rho = torch.full((C_,), 10.0, dtype=torch.float64, device=dev)
    items = (_lib.BatchItem * 1)()
    items[0] = _lib.BatchItem(net.handle.value, C_, Y.data_ptr(), rho.data_ptr(), T.data_ptr(),
                              None, None, None)
    need = L.burn_batch_multi_order_workspace_bytes(1, items)
    assert need > (64 << 20)
    opts = _lib.BurnOpts(0, 0, 0, 1)
    rc = L.burn_batch_multi_noalloc(1, items, 1e-2, 1e-6, 1e-10, C.byref(opts),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.BN_EINVAL
    msg = L.bn_last_error().decode()
    assert "scratch" in msg and str(need) in msg, msg
    torch.cuda.synchronize()
    assert torch.equal(T, torch.full_like(T, 2.0))  # nothing ran
    net.close()
