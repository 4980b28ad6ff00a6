"""Pins of the oracle's burn with a constant per-cell source (the advective
forcing of a simplified-SDC coupling, dy/dt = f(y) + A_adv): exact linear
growth when no reaction can fire, a decay with inflow in closed form, and the
mass invariant with a source."""
import numpy as np

from paper_2312_02836_amd import synth


def _one(Y, rho, T):
    return synth.Cells(np.asarray(Y, dtype=np.float64).reshape(-1, 1), np.array([rho]),
                       np.array([T]))


def test_source_only_is_integrated_exactly(oracle):
    """All abundances zero: no reaction fires until the source has built some
    up.  With a source only on the last species of the chain (a product no
    reaction consumes), f = s exactly, and every BDF order integrates the
    linear-in-time solution to roundoff."""
    spec = synth.chain_network([3.0, 0.7], q=[1.0, 2.0], c_v=10.0)
    net = oracle.OracleNet(spec)
    s = np.array([[0.0], [0.0], [0.4], [0.05]])
    for t_end in (0.1, 3.0):
        Y, T, st, cnt = oracle.burn(net, _one([0.0, 0.0, 0.0], 1.0, 2.0), t_end, source=s)
        assert st[0] == 0
        assert np.allclose(Y[:, 0], [0.0, 0.0, 0.4 * t_end], rtol=1e-13, atol=1e-15)
        assert np.isclose(T[0], 2.0 + 0.05 * t_end, rtol=1e-13)


def test_decay_with_inflow_closed_form(oracle):
    """A -> B at rate k with a constant inflow s of A:
    A(t) = s/k + (A0 - s/k) e^{-kt}, B = A0 + s t - A."""
    k, s_a, A0 = 2.5, 0.3, 1.0
    spec = synth.chain_network([k])
    net = oracle.OracleNet(spec)
    src = np.array([[s_a], [0.0], [0.0]])
    for rtol in (1e-6, 1e-10):
        for t_end in (0.2, 4.0):
            Y, T, st, cnt = oracle.burn(net, _one([A0, 0.0], 1.0, 2.0), t_end, rtol=rtol,
                                        atol=1e-14, source=src)
            a = s_a / k + (A0 - s_a / k) * np.exp(-k * t_end)
            ref = np.array([a, A0 + s_a * t_end - a])
            tol = 100 * rtol * np.abs(ref) + 1e-13
            assert np.all(np.abs(Y[:, 0] - ref) <= tol), (Y[:, 0], ref)


def test_mass_with_source(oracle):
    """sum_i A_i Y_i grows at the constant rate sum_i A_i s_i (the reactions
    conserve it), exactly to roundoff for the BDF."""
    cfg = synth.config(2, n_cells=32)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(9)
    src = np.abs(rng.normal(0.0, 0.5, size=(spec.n, 32)))
    Y, T, st, cnt = oracle.burn(net, cells, cfg.t_end, source=src)
    assert np.all(st == 0)
    A = spec.mass.astype(np.float64)
    m0 = A @ cells.Y
    m1 = A @ Y
    ref = m0 + cfg.t_end * (A @ src[:spec.n_species])
    assert np.allclose(m1, ref, rtol=1e-12, atol=0)
    # and it differs from the burn without a source
    Y2, *_ = oracle.burn(net, cells, cfg.t_end)
    assert np.abs(Y2 - Y).max() > 1e-4
