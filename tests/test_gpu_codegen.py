"""The generated per-network kernels (bn_network_generate) against the CPU
oracle on the same seeded inputs, through the C ABI: element by element on
small, ragged and pivoting cases, on a sample of the full 65,536-cell
workload in the benchmark's launch (ordered persistent queue), inside mixed
multi-network launches and graph replays, and on the failure paths."""
import numpy as np
import pytest

from paper_2312_02836_amd import synth
from tests.parity import assert_parity, gate_for

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-6, 1e-10


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2312_02836_amd import burn as B
    return B


def _host(out):
    import torch
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in out)


def _gen_net(B, spec, lanes=0):
    net = B.Network(spec)
    got = net.generate(lanes)
    assert net.body == ("generated", got)
    if lanes:
        assert got == lanes
    return net


def _check(g, oracle, spec, cells, t_end, rtol=RTOL, atol=ATOL, log_mult=None, label=None,
           max_steps=100000, **gate):
    o = oracle.burn(oracle.OracleNet(spec), cells, t_end, rtol, atol, log_mult=log_mult,
                    max_steps=max_steps)

    def tight(idx):
        r = oracle.burn(oracle.OracleNet(spec), cells.subset(idx), t_end, rtol * 1e-4,
                        atol * 1e-4, log_mult=log_mult)
        return r[0], r[1]

    kw = dict(gate_for(spec))
    kw.update(gate)
    return assert_parity(g, o, rtol, atol, tight=tight, label=label, **kw)


def _small(name):
    return {"chain4": synth.chain_network([3.0, 0.7, 0.05], q=[1.0, 2.0, 0.5]),
            "pair1": synth.reversible_pair(3.0, 0.5),
            "pair2": synth.reversible_pair(2.0, 0.3, two_body=True)}[name]


@pytest.mark.parametrize("name", ["chain4", "pair1", "pair2"])
def test_generated_small_networks(gpu, oracle, name):
    spec = _small(name)
    y0 = np.zeros(spec.n_species)
    y0[0] = 1.0
    cells = synth.draw_cells(5, spec, 300, T_range=(1.0, 3.0), rho_range=(1.0, 10.0), y0=y0)
    net = _gen_net(gpu, spec)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, 5.0, RTOL, ATOL))
    _check(g, oracle, spec, cells, 5.0, label=f"generated {name}")
    net.close()


@pytest.mark.parametrize("lanes", [1, 2])
def test_generated_robertson_both_layouts(gpu, oracle, lanes):
    cfg = synth.config(1)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec, lanes)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL))
    _check(g, oracle, spec, cells, cfg.t_end, label=f"generated robertson, {lanes} lane(s)")
    assert np.all(g[2] == 0)
    net.close()


def test_generated_synth13_ragged(gpu, oracle):
    """4,099 cells of the 13/30 network: every wave of the grid takes cells
    and the last ones are ragged."""
    cfg = synth.config(2, n_cells=4099)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    assert net.body[1] == 2
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL))
    _check(g, oracle, spec, cells, cfg.t_end, label="generated synth13 ragged")
    assert np.all(g[2] == 0)
    net.close()


def test_generated_pivoting_network(gpu, oracle):
    """The mixed workload's 13/30 network: partial pivoting leaves the
    diagonal in about 1.6 % of its factorizations (the rest take the
    compile-time fill pattern), so cells go through the pivoting path and
    its solves."""
    cfg = synth.config(4, n_cells=2048)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL))
    _check(g, oracle, spec, cells, cfg.t_end, label="generated synth13 s44 (pivoting)")
    net.close()


def test_generated_log_multipliers(gpu, oracle):
    cfg = synth.config(2, n_cells=700)
    spec, cells = cfg.networks[0], cfg.cells[0]
    lm = np.random.default_rng(3).normal(0.0, 0.5, spec.n_reactions)
    net = _gen_net(gpu, spec)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL, log_mult=lm))
    _check(g, oracle, spec, cells, cfg.t_end, log_mult=lm, label="generated log multipliers")
    net.close()


def test_generated_tight_tolerance(gpu, oracle):
    cfg = synth.config(2, n_cells=300)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, 1e-9, 1e-14))
    # one-ulp changes of the oracle's own rounding flip 1-2 % of these cells
    # at rtol 1e-9 (tests/test_oracle_rounding.py)
    _check(g, oracle, spec, cells, cfg.t_end, 1e-9, 1e-14, min_counter_equal=0.95,
           label="generated tight tolerance")
    net.close()


def test_generated_failure_paths(gpu, oracle):
    cfg = synth.config(2, n_cells=64)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    bad = synth.Cells(cells.Y.copy(), cells.rho.copy(), cells.T.copy())
    bad.rho[3] = np.nan
    bad.T[5] = 0.0
    bad.T[6] = -1.0
    bad.Y[2, 7] = np.inf
    g = _host(gpu.burn(net, bad.Y, bad.rho, bad.T, cfg.t_end, RTOL, ATOL))
    _check(g, oracle, spec, bad, cfg.t_end)
    assert list(np.nonzero(g[2])[0]) == [3, 5, 6, 7] and np.all(g[2][[3, 5, 6, 7]] == 4)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL, max_steps=3))
    _check(g, oracle, spec, cells, cfg.t_end, max_steps=3)
    assert np.all(g[2] == 1) and np.all(g[3][0] == 3)
    net.close()
    big = synth.NetworkSpec.from_json(spec.to_json())
    big.coef[0, 0] = 800.0
    net = _gen_net(gpu, big)
    g = _host(gpu.burn(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL))
    _check(g, oracle, big, cells, cfg.t_end)
    assert np.all(g[2] == 3)
    net.close()


def test_generated_empty_determinism_and_order(gpu):
    """No cells is a no-op; two runs are bitwise equal; a permuted batch and
    the ordered persistent launch give bitwise the same per-cell results
    (a cell's arithmetic does not depend on where or when it runs)."""
    import torch
    cfg = synth.config(2, n_cells=1024)
    net = _gen_net(gpu, cfg.networks[0])
    c = cfg.cells[0]
    out0 = gpu.burn(net, c.Y[:, :0], c.rho[:0], c.T[:0], cfg.t_end)
    assert out0[0].shape == (13, 0)
    a = _host(gpu.burn(net, c.Y, c.rho, c.T, cfg.t_end))
    b = _host(gpu.burn(net, c.Y, c.rho, c.T, cfg.t_end))
    perm = np.random.default_rng(5).permutation(c.n_cells)
    inv = np.argsort(perm)
    cp = c.subset(perm)
    p = _host(gpu.burn(net, cp.Y, cp.rho, cp.T, cfg.t_end))
    m = _host(gpu.burn_multi([(net, cp.Y, cp.rho, cp.T)], cfg.t_end, order_cells=True)[0])
    torch.cuda.synchronize()
    for x, y, z, w in zip(a, b, p, m):
        assert np.array_equal(x, y)
        assert np.array_equal(x, z[..., inv]) and np.array_equal(x, w[..., inv])
    net.close()


def test_generated_full_size_sampled(gpu, oracle):
    """The benchmark workload (65,536 cells of the 13/30 network) in the
    benchmark's launch (ordered persistent queue, generated kernel); the
    oracle recomputes a seeded sample of 2,048 cells."""
    cfg = synth.config(2)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    out = _host(gpu.burn_multi([(net, cells.Y, cells.rho, cells.T)], cfg.t_end, RTOL, ATOL,
                               order_cells=True)[0])
    idx = np.sort(np.random.default_rng(0).choice(cells.n_cells, 2048, replace=False))
    g = (out[0][:, idx], out[1][idx], out[2][idx], out[3][:, idx])
    _check(g, oracle, spec, cells.subset(idx), cfg.t_end, label="generated synth13 full launch")
    assert np.all(out[2] == 0)
    net.close()


def test_generated_in_mixed_multi_launch(gpu, oracle):
    """A generated network and table-driven ones in one burn_multi call (the
    generated one runs as its own launch, the others share the persistent
    launch): every network matches the oracle."""
    cfg = synth.config(4, n_cells=512)
    nets = []
    for j, spec in enumerate(cfg.networks[:3]):
        net = gpu.Network(spec)
        if j == 0:
            net.generate()
        nets.append(net)
    outs = gpu.burn_multi([(net, c.Y, c.rho, c.T) for net, c in zip(nets, cfg.cells[:3])],
                          cfg.t_end, RTOL, ATOL, order_cells=True)
    for j, (spec, cells, out) in enumerate(zip(cfg.networks[:3], cfg.cells[:3], outs)):
        _check(_host(out), oracle, spec, cells, cfg.t_end,
               label=f"mixed launch, {'generated' if j == 0 else 'table'} {spec.name}")
    for net in nets:
        net.close()


def test_generated_graph_replay(gpu):
    """A MultiBurn with a generated network captured into a HIP graph:
    every replay (with eager work between) equals the eager run bitwise."""
    import torch
    cfg = synth.config(2, n_cells=2048)
    net = _gen_net(gpu, cfg.networks[0])
    c = cfg.cells[0]
    dev = torch.device("cuda", 0)
    Y0, T0 = torch.as_tensor(c.Y, device=dev), torch.as_tensor(c.T, device=dev)
    Yw, Tw = Y0.clone(), T0.clone()
    mb = gpu.MultiBurn([(net, Yw, torch.as_tensor(c.rho, device=dev), Tw)], cfg.t_end, RTOL,
                       ATOL)
    mb.run()
    torch.cuda.synchronize()
    eager = tuple(x.clone() for x in mb.outputs[0][:4])
    mb.capture()
    for rep in range(3):
        Yw.copy_(Y0)
        Tw.copy_(T0)
        torch.cuda.synchronize()
        mb.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=dev).sum()  # eager work between replays
        torch.cuda.synchronize()
        for x, y in zip(mb.outputs[0][:4], eager):
            assert torch.equal(x, y), f"replay {rep} differs"
        del junk
    net.close()


def test_generated_and_table_bodies_agree(gpu):
    """The same cells through both bodies of one network: the generated
    body's sums follow the definitions' order, the table body's do not, so
    the two differ by rounding only: the same status everywhere and the
    decisions of (nearly) every cell."""
    cfg = synth.config(2, n_cells=2048)
    spec, c = cfg.networks[0], cfg.cells[0]
    net = _gen_net(gpu, spec)
    g = _host(gpu.burn(net, c.Y, c.rho, c.T, cfg.t_end, RTOL, ATOL))
    net.set_body("table")
    t = _host(gpu.burn(net, c.Y, c.rho, c.T, cfg.t_end, RTOL, ATOL))
    net.set_body("generated")
    assert np.array_equal(g[2], t[2])
    same = np.all(g[3] == t[3], axis=0)
    assert same.mean() >= 0.999, same.mean()
    y_g, y_t = np.vstack([g[0], g[1]]), np.vstack([t[0], t[1]])
    ewt = np.abs(y_g - y_t) / (RTOL * np.abs(y_t) + ATOL)
    assert ewt[:, same].max() <= 1.0
    net.close()
