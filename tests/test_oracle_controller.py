"""Pins of the oracle's step-size and order controller (the integrator the
paper runs per zone is a VODE-class variable-order BDF, Sec. 2; the oracle's
controller is the quasi-constant-step BDF of Shampine & Reichelt with
kappa = 0 and the Hairer-Norsett-Wanner starting step).

What fixes each part from outside the oracle:
  * the initial step: scipy's implementation of the same published
    starting-step algorithm (HNW vol. I, Sec. II.4) with p = 1;
  * the error estimate C_k ||d||: the leading term of BDF_k's local
    truncation error, (1/(k+1)) h^(k+1) y^(k+1), computed from the exact
    solution of a linear system; and the one-step error itself, which is
    that term divided by gamma_k;
  * the order choice: the estimates of the neighbouring orders are the
    truncation errors of BDF_(k-1) and BDF_(k+1), and the decision rule is
    checked on constructed inputs whose norms are exact powers of two
    (both tie rules, the order limits, the factor clamp);
  * the whole controller: accepted-step counts within a factor 3 of scipy's
    own BDF on the same problems, and orders of 3 and more on smooth phases.

Each pin is a function of the oracle binding, so tests/test_oracle_mutants.py
can run it against builds of the oracle with a planted mistake.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.integrate._ivp.common import select_initial_step

from paper_2312_02836_amd import synth

GAMMA = [0.0] + [sum(1.0 / j for j in range(1, k + 1)) for k in range(1, 7)]


def _wrms(v, s):
    return float(np.sqrt(np.mean((np.asarray(v) / np.asarray(s)) ** 2)))


# ---------------------------------------------------------------------------
# Initial step
# ---------------------------------------------------------------------------

def _initial_step_cases():
    """(spec, rho, y0, t_end, rtol, atol) for the starting-step pins: a
    single decay (y' = -lambda y), a two-species linear system, the
    Robertson-like network and the 13-species network."""
    cases = []
    cases.append((synth.chain_network([4.0]), 1.0, [1.0, 0.0, 1.5], 10.0, 1e-6, 1e-10))
    cases.append((synth.chain_network([4.0]), 1.0, [1.0, 0.0, 1.5], 1e-4, 1e-6, 1e-10))
    cases.append((synth.reversible_pair(3.0, 0.5), 1.0, [0.7, 0.3, 2.0], 5.0, 1e-8, 1e-12))
    c1 = synth.config(1, n_cells=3)
    for i in range(3):
        cells = c1.cells[0]
        cases.append((c1.networks[0], cells.rho[i],
                      np.concatenate([cells.Y[:, i], [cells.T[i]]]), c1.t_end, 1e-6, 1e-10))
    c2 = synth.config(2, n_cells=4)
    for i in range(4):
        cells = c2.cells[0]
        cases.append((c2.networks[0], cells.rho[i],
                      np.concatenate([cells.Y[:, i], [cells.T[i]]]), c2.t_end, 1e-6, 1e-10))
    # a state at rest (every rate zero): d1 = 0, the 1e-6 branch
    cases.append((synth.chain_network([4.0]), 1.0, [0.0, 1.0, 1.5], 1.0, 1e-6, 1e-10))
    # a state far below atol (d0 < 1e-5: h0 = 1e-6) whose slow change allows
    # a large h1, so the step is the cap 100 h0
    cases.append((synth.chain_network([4.0]), 1.0, [1e-16, 0.0, 1e-16], 1.0, 1e-6, 1e-10))
    return cases


def pin_initial_step(O):
    """The oracle's first step equals scipy's select_initial_step with order
    1 on every case (same algorithm, independent code: equal up to the
    rounding of the norms)."""
    for spec, rho, y0, t_end, rtol, atol in _initial_step_cases():
        net = O.OracleNet(spec)
        y0 = np.asarray(y0, dtype=np.float64)
        f0 = O.rhs(net, rho, y0)
        ref = select_initial_step(lambda t, y: O.rhs(net, rho, y), 0.0, y0, t_end, np.inf, f0,
                                  1.0, 1, rtol, atol)
        h = O.initial_step(net, rho, y0, t_end, rtol, atol)
        assert h == pytest.approx(ref, rel=1e-12), (spec.name, h, ref)
        # the integrator starts with exactly this step
        _, st, _, h_init, _, _, _ = O.burn_cell_schedule(net, rho, y0, t_end, rtol, atol,
                                                           max_steps=2)
        assert h_init == h


def test_initial_step_matches_hnw_reference(oracle):
    pin_initial_step(oracle)


# ---------------------------------------------------------------------------
# Error estimate of an order-k step
# ---------------------------------------------------------------------------

# the linear test problem: A -> B -> C with temperature-independent rates
K1, K2 = 1.0, 2.0
A_MAT = np.array([[-K1, 0.0, 0.0, 0.0],
                  [K1, -K2, 0.0, 0.0],
                  [0.0, K2, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0]])


def _exact(t):
    a = math.exp(-K1 * t)
    b = K1 / (K2 - K1) * (math.exp(-K1 * t) - math.exp(-K2 * t))
    return np.array([a, b, 1.0 - a - b, 1.0])


def _exact_history(k, h):
    """Backward differences D_0..D_k of the exact solution at t = 0, -h, ...,
    -k h (by their definition: alternating binomial sums of the values)."""
    vals = [_exact(-m * h) for m in range(k + 1)]
    return np.array([sum(((-1) ** m) * math.comb(j, m) * vals[m] for m in range(j + 1))
                     for j in range(k + 1)])


def _one_step(O, k, h):
    net = O.OracleNet(synth.chain_network([K1, K2]))
    D = _exact_history(k, h)
    y_new, st, cnt = O.burn_fixed(net, 1.0, D, k, h, 1, newton_tol=1e-14)
    assert st == 1 and cnt[0] == 1
    return D, y_new


def _deriv(m, t):
    """m-th derivative of the exact solution: A^m y(t)."""
    return np.linalg.matrix_power(A_MAT, m) @ _exact(t)


def _grad_exact(j, h):
    """j-th backward difference of the exact solution at t = h (step h)."""
    return sum(((-1) ** m) * math.comb(j, m) * _exact(h - m * h) for m in range(j + 1))


def pin_error_estimate(O):
    """The error constant: applied to the (k+1)-th backward difference of
    the exact solution, the estimator gives the norm of BDF_k's truncation
    error, i.e. of the residual tau = sum_{j<=k} (1/j) grad^j y(h) - h y'(h)
    of the formula on the exact solution (ratio -> 1 as h -> 0).  And on a
    real step, where d = y_new - y_pred = e + grad^(k+1) y(h) with the
    one-step error e = y_new - y(h) ~ -tau / gamma_k, the estimate is
    (gamma_k + 1/(k+1)) ||e|| to leading order."""
    rtol, atol = 1e-6, 1e-12
    for k in range(1, 6):
        dev = []
        for h in (0.02, 0.005):
            tau = sum(_grad_exact(j, h) / j for j in range(1, k + 1)) - h * (A_MAT @ _exact(h))
            err, s = O.error_norm(k, _grad_exact(k + 1, h), _exact(0.0), _exact(h), rtol, atol)
            np.testing.assert_array_equal(
                s, atol + rtol * np.maximum(np.abs(_exact(0.0)), np.abs(_exact(h))))
            dev_tau = abs(err / _wrms(tau, s) - 1.0)
            D, y_new = _one_step(O, k, h)
            d = y_new - D.sum(axis=0)
            err_step, s_step = O.error_norm(k, d, D[0], y_new, rtol, atol)
            ratio = err_step / _wrms(y_new - _exact(h), s_step)
            dev.append((dev_tau, abs(ratio / (GAMMA[k] + 1.0 / (k + 1)) - 1.0)))
        (d_big, e_big), (d_small, e_small) = dev
        assert d_small < 0.05 and d_small < d_big, (k, dev)
        assert e_small < 0.05 and e_small < e_big, (k, dev)


def test_error_estimate_is_the_truncation_error(oracle):
    pin_error_estimate(oracle)


def _bdf_residual(q, h):
    """Truncation error of BDF_q at t = h: the residual of the formula
    sum_{j<=q} (1/j) grad^j y - h y' on the exact solution."""
    return sum(_grad_exact(j, h) / j for j in range(1, q + 1)) - h * (A_MAT @ _exact(h))


def pin_neighbour_order_estimates(O):
    """The order choice's estimates for the neighbouring orders: given the
    rows D_k = grad^k y and D_(k+2) = grad^(k+2) y of the exact solution,
    the step ratio it returns when order k-1 (k+1) is chosen is
    0.9 e^(-1/k) (0.9 e^(-1/(k+2))) with e the truncation error of BDF_(k-1)
    (BDF_(k+1)); the estimate recovered from the ratio converges to that
    error as h -> 0."""
    for k in (2, 3, 4):
        dev = []
        for h in (0.04, 0.01):
            dk, dk2 = _grad_exact(k, h), _grad_exact(k + 2, h)
            big = np.full(4, 1e30)
            # order k-1 wins (order k and k+1 estimates made huge)
            s = np.full(4, _wrms(_bdf_residual(k - 1, h), np.ones(4)))
            kn, f = O.choose_order(k, 1e30, dk, big, s)
            assert kn == k - 1
            e_low = (f / 0.9) ** (-k)
            # order k+1 wins
            s = np.full(4, _wrms(_bdf_residual(k + 1, h), np.ones(4)))
            kn, f = O.choose_order(k, 1e30, big, dk2, s)
            assert kn == k + 1
            e_high = (f / 0.9) ** (-(k + 2))
            dev.append(max(abs(e_low - 1.0), abs(e_high - 1.0)))
        assert dev[1] < 0.08 and dev[1] < dev[0], (k, dev)


def test_neighbour_order_estimates(oracle):
    pin_neighbour_order_estimates(oracle)


def pin_order_choice_rules(O):
    """The decision rule on inputs whose norms are exact: unit scales and
    rows whose weighted RMS norms, after the divisions by k and k+2, are the
    chosen powers of two, so each order's step ratio is an exact power of
    two.  SAFETY = 0.9, MAX_FACTOR = 10."""
    n = 5
    s = np.ones(n)

    def rows(k, em, ep):
        return np.full(n, k * em), np.full(n, (k + 2) * ep)

    k = 3
    # all three ratios 1: keep k, factor 0.9
    assert O.choose_order(k, 1.0, *rows(k, 1.0, 1.0), s) == (3, pytest.approx(0.9, rel=1e-15))
    # k-1 and k+1 tie above k: the lower order wins
    kn, f = O.choose_order(k, 2.0 ** 4, *rows(k, 1.0, 1.0), s)
    assert (kn, f) == (2, pytest.approx(0.9, rel=1e-15))
    # k and k+1 tie above k-1: k stays
    kn, f = O.choose_order(k, 1.0, *rows(k, 2.0 ** 3, 1.0), s)
    assert (kn, f) == (3, pytest.approx(0.9, rel=1e-15))
    # k-1 and k tie (ratio 2) above k+1: k stays, factor 1.8
    kn, f = O.choose_order(k, 2.0 ** -4, *rows(k, 2.0 ** -3, 1.0), s)
    assert (kn, f) == (3, pytest.approx(1.8, rel=1e-14))
    # k+1 strictly best (ratio 2)
    kn, f = O.choose_order(k, 1.0, *rows(k, 1.0, 2.0 ** -5), s)
    assert (kn, f) == (4, pytest.approx(1.8, rel=1e-14))
    # k-1 strictly best (ratio 4)
    kn, f = O.choose_order(k, 1.0, *rows(k, 2.0 ** -6, 1.0), s)
    assert (kn, f) == (2, pytest.approx(3.6, rel=1e-14))
    # a tiny error allows more than MAX_FACTOR: clamped to 10
    kn, f = O.choose_order(k, 1e-30, *rows(k, 1.0, 1.0), s)
    assert (kn, f) == (3, 10.0)
    # a zero error: infinite ratio, k stays, clamped
    kn, f = O.choose_order(k, 0.0, *rows(k, 1.0, 1.0), s)
    assert (kn, f) == (3, 10.0)
    # order 1 has no lower order, however small its row
    kn, f = O.choose_order(1, 1.0, np.zeros(n), np.full(n, 3.0), s)
    assert (kn, f) == (1, pytest.approx(0.9, rel=1e-15))
    # order 5 has no higher order, however small its row
    kn, f = O.choose_order(5, 1.0, np.full(n, 5.0), np.zeros(n), s)
    assert (kn, f) == (5, pytest.approx(0.9, rel=1e-15))
    # the norm is the weighted RMS: one component of four at 2 gives 1
    s4 = np.array([1.0, 2.0, 4.0, 8.0])
    dk = np.array([0.0, 0.0, 0.0, 2 * 8.0 * 2.0])   # (dk/2)/s = (0, 0, 0, 2): RMS 1
    dk2 = np.full(4, 4 * 1.0) * s4                  # (dk2/4)/s = 1: RMS 1
    kn, f = O.choose_order(2, 2.0 ** 3, dk, dk2, s4)  # ratios 1, 1/2, 1: tie k-1, k+1
    assert (kn, f) == (1, pytest.approx(0.9, rel=1e-15))


def test_order_choice_rules(oracle):
    pin_order_choice_rules(oracle)


# ---------------------------------------------------------------------------
# The whole controller against an independent BDF
# ---------------------------------------------------------------------------

def _controller_cells():
    out = []
    c1 = synth.config(1, n_cells=64)
    for i in (0, 17, 40, 63):
        cells = c1.cells[0]
        out.append((c1.networks[0], cells.rho[i], np.concatenate([cells.Y[:, i], [cells.T[i]]]),
                    c1.t_end))
    c2 = synth.config(2, n_cells=2048)
    for i in (0, 1, 2, 3, 100, 500, 1000, 2047):
        cells = c2.cells[0]
        out.append((c2.networks[0], cells.rho[i], np.concatenate([cells.Y[:, i], [cells.T[i]]]),
                    c2.t_end))
    out.append((synth.chain_network([K1, K2]), 1.0, [1.0, 0.0, 0.0, 1.0], 20.0))
    return out


def pin_step_counts_vs_scipy_bdf(O):
    """Accepted steps within a factor 3 of scipy's BDF (Shampine & Reichelt's
    variable-order quasi-constant-step scheme with its default NDF
    coefficients) at the same tolerances, and a maximum order of at least 3
    over the run (the solutions have smooth phases)."""
    rtol, atol = 1e-6, 1e-10
    ratios = []
    for spec, rho, y0, t_end in _controller_cells():
        net = O.OracleNet(spec)
        y0 = np.asarray(y0, dtype=np.float64)
        y, st, cnt, h_init, h, ratio, order = O.burn_cell_schedule(net, rho, y0, t_end, rtol,
                                                                    atol)
        assert st == 0
        sol = solve_ivp(lambda t, yy: O.rhs(net, rho, yy), (0.0, t_end), y0, method="BDF",
                        rtol=rtol, atol=atol, jac=lambda t, yy: O.jac(net, rho, yy))
        assert sol.success
        n_ref = len(sol.t) - 1
        ratios.append(cnt[0] / n_ref)
        assert 1.0 / 3.0 <= cnt[0] / n_ref <= 3.0, (spec.name, cnt[0], n_ref)
        assert order.max() >= 3, (spec.name, np.bincount(order))
        assert len(h) == cnt[0] and np.all(h > 0) and abs(h.sum() - t_end) <= 1e-12 * t_end
    return ratios


def test_step_counts_vs_scipy_bdf(oracle):
    pin_step_counts_vs_scipy_bdf(oracle)


def _scipy_bdf_kappa0(O, net, rho, y0, t_end, rtol, atol):
    """scipy's BDF (Shampine & Reichelt's scheme, independent code) set to
    the coefficients of the plain BDFs (kappa = 0: alpha_k = gamma_k, error
    constants 1/(k+1)) and the Newton tolerance 0.03.  What still differs
    from the oracle's scheme: its safety factor 0.9 * 9 / (8 + Newton
    iterations) (<= 0.9), the error scale atol + rtol |y_new|, ties in the
    order choice going to the lowest order, and no new LU after a rejected
    step.  Returns the order of every accepted step."""
    from scipy.integrate._ivp.bdf import BDF
    s = BDF(lambda t, y: O.rhs(net, rho, y), 0.0, np.array(y0, dtype=np.float64), t_end,
            rtol=rtol, atol=atol, jac=lambda t, y: O.jac(net, rho, y))
    s.alpha = s.gamma.copy()
    s.error_const = 1.0 / np.arange(1, 7)
    s.newton_tol = 0.03
    orders = []
    while s.status == "running":
        s.step()
        orders.append(s.order)
    assert s.status == "finished"
    return np.array(orders)


def pin_order_usage_vs_scipy_kappa0(O):
    """Against scipy's BDF with the same coefficients: per cell at most 5 %
    more accepted steps (its safety factor is never larger, so it takes more
    steps, not fewer: observed 6-10 % more than the oracle) and in total
    between 0 and 15 % fewer; the step-weighted mean order within 0.3 per
    cell and 0.15 overall.  An order choice that reads the wrong history
    row or divides by the wrong constants changes both."""
    rtol, atol = 1e-6, 1e-10
    n_o = n_s = 0
    ord_o = ord_s = 0.0
    for spec, rho, y0, t_end in _controller_cells():
        net = O.OracleNet(spec)
        _, st, cnt, _, _, _, order = O.burn_cell_schedule(net, rho, y0, t_end, rtol, atol)
        assert st == 0
        ref = _scipy_bdf_kappa0(O, net, rho, y0, t_end, rtol, atol)
        assert len(order) <= 1.05 * len(ref), (spec.name, len(order), len(ref))
        assert abs(order.mean() - ref.mean()) <= 0.3, (spec.name, order.mean(), ref.mean())
        n_o += len(order)
        n_s += len(ref)
        ord_o += order.sum()
        ord_s += ref.sum()
    assert 0.85 * n_s <= n_o <= n_s, (n_o, n_s)
    assert abs(ord_o / n_o - ord_s / n_s) <= 0.15, (ord_o / n_o, ord_s / n_s)


def test_order_usage_vs_scipy_kappa0(oracle):
    pin_order_usage_vs_scipy_kappa0(oracle)


def pin_smooth_problem_reaches_order_5(O):
    """On a smooth linear problem at a tight tolerance the controller climbs
    to the highest order and stays there: each order change needs k+1 steps
    at constant h and a larger allowed step at the new order, so the orders
    of the accepted steps never fall during the climb and the last fifth of
    the steps run at order 5."""
    net = O.OracleNet(synth.chain_network([K1, K2]))
    y, st, cnt, h_init, h, ratio, order = O.burn_cell_schedule(net, 1.0, [1.0, 0.0, 0.0, 1.0],
                                                                30.0, 1e-10, 1e-14)
    assert st == 0
    first5 = int(np.argmax(order == 5))
    assert order[first5] == 5
    assert np.all(np.diff(order[:first5 + 1]) >= 0), order[:first5 + 1]
    tail = order[-max(1, len(order) // 5):]
    assert np.all(tail == 5), np.bincount(order)
    # the rescale product of a step taken right after an order change is the
    # step ratio that change chose, which is at most MAX_FACTOR
    assert np.all(ratio <= 10.0 + 1e-12)


def test_smooth_problem_reaches_order_5(oracle):
    pin_smooth_problem_reaches_order_5(oracle)
