"""Pins of the oracle's forward sensitivities S = d y_end / d p (p = log-rate
multipliers) of the burn replayed on its frozen schedule with exact
correctors: central finite differences of that same replay, closed forms of
a decay chain and of an equilibrium, and the linear mass invariant."""
import numpy as np
import pytest

from paper_2312_02836_amd import synth


def _cells(spec, n, seed=3, T=(1.0, 3.0), y0=None):
    if y0 is None:
        y0 = np.zeros(spec.n_species)
        y0[0] = 1.0
    return synth.draw_cells(seed, spec, n, T_range=T, rho_range=(1.0, 10.0), y0=y0)


@pytest.mark.parametrize("h", [1e-4, 1e-6])
def test_sens_matches_central_differences_of_the_replay(oracle, h):
    """Finite differences of the frozen-schedule replay (the schedule is
    recorded once at p = 0 and replayed at +-h e_r) against S, for every
    reaction, on the 21-species / 60-reaction network, at the step 1e-6 the
    sensitivity workload names and at 1e-4.  The difference error is the
    replay's rounding noise / h (about 3e-14 |y| / h here) plus O(h^2), so
    the bound is 1e-6 of the column's scale plus that noise floor."""
    cfg = synth.config(5, n_cells=24)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    Y, T, st, cnt, S, unc = oracle.sens(net, cells, cfg.t_end)
    assert np.all(st == 0) and np.all(unc == 0)
    y = np.vstack([Y, T[None]])
    for r in range(spec.n_reactions):
        e = np.zeros(spec.n_reactions)
        e[r] = h
        Yp, Tp, *_ = oracle.sens(net, cells, cfg.t_end, log_mult_replay=e, want_S=False)
        Ym, Tm, *_ = oracle.sens(net, cells, cfg.t_end, log_mult_replay=-e, want_S=False)
        fd = (np.vstack([Yp, Tp[None]]) - np.vstack([Ym, Tm[None]])) / (2 * h)
        an = S[:, :, r].T
        bound = 1e-6 * np.abs(an).max(axis=0, keepdims=True) + 1e-13 * np.maximum(np.abs(y), 1.0) / h
        assert np.all(np.abs(fd - an) <= bound), (r, np.abs(fd - an).max())


def _bateman_sens(k1, k2, t):
    """A, B, C of A -> B -> C and their derivatives with respect to ln k1,
    ln k2 (closed form)."""
    e1, e2 = np.exp(-k1 * t), np.exp(-k2 * t)
    A = e1
    B = k1 / (k2 - k1) * (e1 - e2)
    dA = np.array([-k1 * t * e1, 0.0])
    dB_dk1 = k2 / (k2 - k1) ** 2 * (e1 - e2) - k1 / (k2 - k1) * t * e1
    dB_dk2 = -k1 / (k2 - k1) ** 2 * (e1 - e2) + k1 / (k2 - k1) * t * e2
    dB = np.array([k1 * dB_dk1, k2 * dB_dk2])
    return A, B, 1.0 - A - B, dA, dB, -dA - dB


def test_sens_bateman_chain_closed_form(oracle):
    """A -> B -> C with heat: the discrete sensitivities at tight tolerance
    against the exact d(A, B, C, T)/d ln k (the discrete map converges to the
    continuous one as rtol -> 0)."""
    k1, k2, q1, q2, cv = 3.0, 0.7, 1.5, 2.5, 10.0
    spec = synth.chain_network([k1, k2], q=[q1, q2], c_v=cv)
    net = oracle.OracleNet(spec)
    cells = synth.Cells(np.array([[1.0], [0.0], [0.0]]), np.array([1.0]), np.array([2.0]))
    for t_end in (0.3, 2.0):
        Y, T, st, cnt, S, unc = oracle.sens(net, cells, t_end, rtol=1e-10, atol=1e-14)
        assert st[0] == 0
        A, B, Cc, dA, dB, dC = _bateman_sens(k1, k2, t_end)
        dT = (-q1 * dA + q2 * dC) / cv
        ref = np.vstack([dA, dB, dC, dT])
        assert np.allclose(S[0], ref, rtol=1e-6, atol=1e-9), (S[0], ref)


def test_sens_equilibrium_closed_form(oracle):
    """A <-> B run to equilibrium: Y_B = K / (1 + K), K = k_f / k_r, so
    dY_B / d ln k_f = -dY_B / d ln k_r = Y_A Y_B, and Y_A's are the negatives."""
    kf, kr = 3.0, 0.5
    spec = synth.reversible_pair(kf, kr)
    net = oracle.OracleNet(spec)
    cells = synth.Cells(np.array([[1.0], [0.0]]), np.array([1.0]), np.array([1.5]))
    Y, T, st, cnt, S, unc = oracle.sens(net, cells, 30.0, rtol=1e-10, atol=1e-14)
    assert st[0] == 0
    ya, yb = kr / (kf + kr), kf / (kf + kr)
    g = ya * yb
    ref = np.array([[-g, g], [g, -g], [0.0, 0.0]])
    assert np.allclose(S[0], ref, rtol=1e-6, atol=1e-9), (S[0], ref)


@pytest.mark.parametrize("cfg_i", [2, 5])
def test_sens_conserves_mass(oracle, cfg_i):
    """sum_i A_i Y_i does not depend on any rate, so sum_i A_i S_ir = 0 for
    every reaction, to the roundoff accumulated over the steps on the scale
    of the cell's sensitivities (a wrong stoichiometric term in df/dp gives
    an O(1) residual)."""
    cfg = synth.config(cfg_i, n_cells=16)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    Y, T, st, cnt, S, unc = oracle.sens(net, cells, cfg.t_end)
    assert np.all(st == 0)
    A = spec.mass.astype(np.float64)
    total = np.einsum("i,cir->cr", A, S[:, :spec.n_species, :])
    scale = np.einsum("i,cir->cr", A, np.abs(S[:, :spec.n_species, :]))
    assert np.all(np.abs(total) <= 1e-11 * scale.max(axis=1, keepdims=True))


def test_replay_close_to_the_burn(oracle):
    """The replay (exact correctors) and the recorded burn (modified Newton
    to tolerance 0.03) are two solutions of the same schedule: within the
    pinned global-error bound of each other."""
    cfg = synth.config(5, n_cells=64)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    Y, T, st, cnt, S, unc = oracle.sens(net, cells, cfg.t_end, want_S=False)
    Yb, Tb, stb, cntb = oracle.burn(net, cells, cfg.t_end)
    assert np.array_equal(st, stb) and np.array_equal(cnt, cntb)
    a, b = np.vstack([Y, T[None]]), np.vstack([Yb, Tb[None]])
    assert np.all(np.abs(a - b) <= 100 * (1e-6 * np.abs(b) + 1e-10))


def test_vjp_is_the_contraction_of_S(oracle):
    cfg = synth.config(5, n_cells=8)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    Y, T, st, cnt, S, unc = oracle.sens(net, cells, cfg.t_end)
    rng = np.random.default_rng(0)
    gY, gE = rng.normal(size=(spec.n_species, 8)), rng.normal(size=8)
    g = oracle.vjp(net, S, gY, gE)
    for c in range(8):
        ref = gY[:, c] @ S[c, :spec.n_species] + gE[c] * spec.c_v * S[c, spec.n_species]
        assert np.allclose(g[:, c], ref, rtol=1e-14, atol=0)


def test_sens_matches_continuous_sensitivities(oracle):
    """The discrete sensitivities at tight tolerance (rtol 1e-8) against the
    continuous ones of the 13-species / 30-reaction network, computed by the
    staggered direct method: scipy's Radau for y (rtol 1e-12, dense output),
    then for every multiplier the linear system s' = J(y(t)) s + df/dp_r
    (rtol 1e-10).  df/dp_r = W_r R_r is a central difference of the oracle's
    RHS in p_r (f is linear in e^{p_r}).  The discrete map converges to the
    continuous one as rtol -> 0: the difference is O(rtol) of the largest
    sensitivity (about 1e-7 of it here)."""
    from scipy.integrate import solve_ivp
    cfg = synth.config(2, n_cells=16)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = oracle.OracleNet(spec)
    R, n = spec.n_reactions, spec.n
    idx = np.array([9, 3])
    sub = cells.subset(idx)
    Yd, Td, st, cnt, S, unc = oracle.sens(net, sub, cfg.t_end, 1e-8, 1e-12)
    assert np.all(st == 0)
    hp = 1e-6
    for c in range(len(idx)):
        rho = sub.rho[c]
        y0 = np.concatenate([sub.Y[:, c], [sub.T[c]]])
        sy = solve_ivp(lambda t, y: oracle.rhs(net, rho, y), (0.0, cfg.t_end), y0,
                       method="Radau", rtol=1e-12, atol=1e-16,
                       jac=lambda t, y: oracle.jac(net, rho, y), dense_output=True)
        assert sy.success
        Sc = np.zeros((n, R))
        for r in range(R):
            e = np.zeros(R)
            e[r] = hp

            def g(t, s, e=e):
                y = sy.sol(t)
                fp = (oracle.rhs(net, rho, y, log_mult=e) - oracle.rhs(net, rho, y, log_mult=-e)) / (2 * hp)
                return oracle.jac(net, rho, y) @ s + fp

            ss = solve_ivp(g, (0.0, cfg.t_end), np.zeros(n), method="Radau", rtol=1e-10, atol=1e-14,
                           jac=lambda t, s: oracle.jac(net, rho, sy.sol(t)))
            assert ss.success
            Sc[:, r] = ss.y[:, -1]
        big = np.abs(Sc).max()
        d = np.abs(S[c] - Sc)
        print(f"cell {idx[c]}: max |S_discrete - S_continuous| = {d.max() / big:.2e} of max |S|")
        assert d.max() <= 1e-5 * big
        assert np.all(d <= 1e-4 * np.abs(Sc).max(axis=0, keepdims=True) + 1e-6 * big)
