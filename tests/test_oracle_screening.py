"""Pins of the oracle's synthetic screening, F_r = exp(h_r G) with
G = sqrt(rho (1 + sum_j A_j^2 Y_j)) T^(-3/2): the factor itself by hand, the
Jacobian's extra composition and temperature terms against finite
differences, mass conservation, the unscreened limit, and an independent
stiff integrator on the screened ODE."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2312_02836_amd import synth
from tests.test_oracle_pins import _fd_jac


def test_screening_factor_by_hand(oracle):
    """2A -> B (A mass 1, B mass 2): f_A = -2 R, R = k e^{hG} rho Y_A^2 / 2."""
    spec = synth.reversible_pair(2.0, 1e-300, two_body=True)
    spec.coef[1, 0] = -700.0  # switch the reverse reaction off
    spec = synth.NetworkSpec("s", spec.mass, spec.reactants, spec.products, spec.coef, spec.q,
                             spec.c_v, np.array([0.05, 0.0]))
    net = oracle.OracleNet(spec)
    rho, ya, yb, T = 3.0, 0.4, 0.2, 1.7
    f = oracle.rhs(net, rho, [ya, yb, T])
    G = math.sqrt(rho * (1.0 + 1.0 * ya + 4.0 * yb)) / T ** 1.5
    R = 2.0 * math.exp(0.05 * G) * rho * ya * ya / 2.0
    assert f[0] == pytest.approx(-2.0 * R, rel=1e-14)
    assert f[1] == pytest.approx(R, rel=1e-14)


@pytest.mark.parametrize("cfg", [2, 5])
def test_screened_jacobian_vs_finite_differences(oracle, cfg):
    spec = synth.screened(synth.config(cfg, n_cells=4).networks[0], 0.01)
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(cfg)
    for _ in range(4):
        y = np.concatenate([rng.uniform(0.01, 1, spec.n_species), [rng.uniform(1.2, 4.5)]])
        rho = 10 ** rng.uniform(0, 2)
        J = oracle.jac(net, rho, y)
        Jfd = _fd_jac(oracle, net, rho, y)
        scale = np.abs(J).max()
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-8 * scale)
        # the screening terms make columns dense: a species column that the
        # unscreened Jacobian leaves empty is now filled
        J0 = oracle.jac(oracle.OracleNet(synth.config(cfg, n_cells=4).networks[0]), rho, y)
        assert np.count_nonzero(J) > np.count_nonzero(J0)


def test_screening_off_is_identical(oracle):
    cfg = synth.config(2, n_cells=16)
    base = cfg.networks[0]
    zero = synth.screened(base, 0.0)
    a = oracle.burn(oracle.OracleNet(base), cfg.cells[0], cfg.t_end)
    b = oracle.burn(oracle.OracleNet(zero), cfg.cells[0], cfg.t_end)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_screened_burn_conserves_mass_and_differs(oracle):
    cfg = synth.config(2, n_cells=32)
    spec = synth.screened(cfg.networks[0])
    Y, T, st, cnt = oracle.burn(oracle.OracleNet(spec), cfg.cells[0], cfg.t_end)
    assert np.all(st == 0)
    A = spec.mass.astype(np.float64)
    m0, m1 = A @ cfg.cells[0].Y, A @ Y
    assert np.allclose(m1, m0, rtol=1e-12, atol=0)
    Y0, *_ = oracle.burn(oracle.OracleNet(cfg.networks[0]), cfg.cells[0], cfg.t_end)
    assert np.abs(Y - Y0).max() > 1e-5


def test_screened_burn_vs_scipy_radau(oracle):
    cfg = synth.config(2, n_cells=8)
    spec = synth.screened(cfg.networks[0])
    net = oracle.OracleNet(spec)
    cells = cfg.cells[0]
    for i in range(0, 8, 3):
        y0 = np.concatenate([cells.Y[:, i], [cells.T[i]]])
        rho = cells.rho[i]
        sol = solve_ivp(lambda t, y: oracle.rhs(net, rho, y), (0.0, cfg.t_end), y0,
                        method="Radau", rtol=1e-12, atol=1e-20,
                        jac=lambda t, y: oracle.jac(net, rho, y))
        assert sol.success
        ref = sol.y[:, -1]
        y, st, _ = oracle.burn_cell(net, rho, y0, cfg.t_end, rtol=1e-10, atol=1e-14)
        assert st == 0
        assert np.all(np.abs(y - ref) <= 1e-7 * np.abs(ref) + 1e-11)
