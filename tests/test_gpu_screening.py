"""Networks with the synthetic screening factor on the GPU, through the C
ABI, against the oracle; the entry points that do not support screening
refuse it."""
import numpy as np
import pytest

from paper_2312_02836_amd import synth
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-6, 1e-10


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2312_02836_amd import burn as B
    return B


@pytest.mark.parametrize("cfg_i,which,C,lanes", [(2, 0, 513, 0), (2, 0, 200, 16), (5, 0, 130, 0),
                                                 (4, 3, 40, 0)])
def test_screened_parity(gpu, oracle, cfg_i, which, C, lanes):
    import torch
    cfg = synth.config(cfg_i, n_cells=C)
    spec = synth.screened(cfg.networks[which])
    cells = cfg.cells[which]
    net = gpu.Network(spec)
    out = gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL, lanes_per_cell=lanes)
    torch.cuda.synchronize()
    g = tuple(x.cpu().numpy() for x in out)
    onet = oracle.OracleNet(spec)
    o = oracle.burn(onet, cells, cfg.t_end, RTOL, ATOL)

    def tight(idx):
        r = oracle.burn(onet, cells.subset(idx), cfg.t_end, RTOL * 1e-4, ATOL * 1e-4)
        return r[0], r[1]

    assert_parity(g, o, RTOL, ATOL, tight=tight)
    assert np.all(g[2] == 0)
    net.close()


def test_screened_unsupported_entry_points(gpu):
    import ctypes as C
    import torch
    from paper_2312_02836_amd import _lib
    cfg = synth.config(5, n_cells=8)
    spec = synth.screened(cfg.networks[0])
    cells = cfg.cells[0]
    net = gpu.Network(spec)
    with pytest.raises(_lib.BurnError, match="screened"):
        gpu.burn_multi([(net, cells.Y, cells.rho, cells.T)], cfg.t_end)
    with pytest.raises(_lib.BurnError, match="screened"):
        gpu.autotune(net, cells.Y, cells.rho, cells.T, cfg.t_end)
    with pytest.raises(_lib.BurnError, match="screened"):
        run = gpu.AdjointRun(net, cells.Y, cells.rho, cells.T, cfg.t_end, max_steps=64)
        run.forward()
    with pytest.raises(_lib.BurnError, match="screened"):
        gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, source=np.zeros((spec.n, 8)))
    torch.cuda.synchronize()
    net.close()
