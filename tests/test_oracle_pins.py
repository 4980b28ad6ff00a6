"""Pins of the CPU oracle against things other than itself: closed forms,
invariants, LAPACK, mpmath at 50 digits and finite differences.

Each test names the part of the oracle it pins and a plausible mistake it
would catch."""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg

from paper_2312_02836_amd import synth

mpmath.mp.dps = 50


def _single_rate_net(coef):
    """A -> B with the given 7 coefficients (T-dependent rate)."""
    c = np.zeros((1, 7))
    c[0] = coef
    return synth.NetworkSpec("one", np.array([1, 1]), np.array([[0, -1, -1]]),
                             np.array([[1, -1, -1]]), c, np.array([0.0]), 100.0)


# ---------------------------------------------------------------------------
# Rates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k,fn", [
    (1, lambda T: math.exp(1.0 / T)),
    (2, lambda T: math.exp(T ** (-1.0 / 3.0))),
    (3, lambda T: math.exp(T ** (1.0 / 3.0))),
    (4, lambda T: math.exp(T)),
    (5, lambda T: math.exp(T ** (5.0 / 3.0))),
    (6, lambda T: T),                 # exp(ln T) = T
])
def test_rate_basis_functions(oracle, k, fn):
    """Each basis slot alone reproduces its textbook function (catches a
    permuted basis or a wrong exponent)."""
    coef = np.zeros(7)
    coef[k] = 1.0
    net = oracle.OracleNet(_single_rate_net(coef))
    for T in (0.7, 1.0, 2.5, 5.0):
        lam, _ = oracle.rates(net, T)
        assert lam[0] == pytest.approx(fn(T), rel=1e-14)


def test_rate_constant_and_multiplier(oracle):
    coef = np.zeros(7)
    coef[0] = math.log(3.5)
    net = oracle.OracleNet(_single_rate_net(coef))
    lam, dl = oracle.rates(net, 2.0)
    assert lam[0] == pytest.approx(3.5, rel=1e-15) and dl[0] == 0.0
    lam, _ = oracle.rates(net, 2.0, log_mult=[math.log(2.0)])
    assert lam[0] == pytest.approx(7.0, rel=1e-15)


def test_rates_vs_mpmath(oracle):
    """lambda and d ln lambda/dT of the config-2 network against the same
    fit evaluated in 50-digit arithmetic (FP64 error bound)."""
    spec = synth.config(2, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    for T in (1.0, 1.37, 2.9, 4.99):
        lam, dl = oracle.rates(net, T)
        Tm = mpmath.mpf(T)
        for r in range(spec.n_reactions):
            a = [mpmath.mpf(float(x)) for x in spec.coef[r]]
            t13 = mpmath.cbrt(Tm)
            expo = (a[0] + a[1] / Tm + a[2] / t13 + a[3] * t13 + a[4] * Tm + a[5] * Tm * t13 ** 2
                    + a[6] * mpmath.log(Tm))
            d = (-a[1] / Tm ** 2 - a[2] / (3 * t13 * Tm) + a[3] * t13 / (3 * Tm) + a[4]
                 + 5 * a[5] * t13 ** 2 / 3 + a[6] / Tm)
            cond = max(1.0, abs(float(expo)))
            assert abs(lam[r] - float(mpmath.exp(expo))) <= 4e-16 * cond * float(mpmath.exp(expo))
            assert abs(dl[r] - float(d)) <= 1e-14 * max(1.0, abs(float(d)))


def test_dlnlam_dT_finite_difference(oracle):
    """The analytic d ln lambda / dT against a central difference of ln lambda."""
    spec = synth.config(5, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    T, h = 2.3, 1e-5
    _, dl = oracle.rates(net, T)
    lp, _ = oracle.rates(net, T + h)
    lm, _ = oracle.rates(net, T - h)
    fd = (np.log(lp) - np.log(lm)) / (2 * h)
    np.testing.assert_allclose(dl, fd, rtol=1e-7, atol=1e-8)


# ---------------------------------------------------------------------------
# Right-hand side
# ---------------------------------------------------------------------------

def test_rhs_chain_closed_form(oracle):
    """Bateman chain s0 -> s1 -> s2 -> s3: f is the textbook linear system."""
    k = [2.0, 0.5, 3.0]
    q = [1.0, 2.0, 4.0]
    net = oracle.OracleNet(synth.chain_network(k, q=q, c_v=10.0))
    y = np.array([0.4, 0.3, 0.2, 0.1, 1.7])
    f = oracle.rhs(net, 5.0, y)
    exp = np.array([-k[0] * y[0], k[0] * y[0] - k[1] * y[1], k[1] * y[1] - k[2] * y[2], k[2] * y[2],
                    (q[0] * k[0] * y[0] + q[1] * k[1] * y[1] + q[2] * k[2] * y[2]) / 10.0])
    np.testing.assert_allclose(f, exp, rtol=1e-15)


def test_rhs_two_body_convention(oracle):
    """2A -> B carries rho^(2-1) and 1/2! (identical-particle factor):
    R = k rho Y_A^2 / 2, f_A = -2R, f_B = R."""
    net = oracle.OracleNet(synth.reversible_pair(4.0, 1.0, two_body=True))
    y = np.array([0.6, 0.2, 1.0])
    rho = 7.0
    f = oracle.rhs(net, rho, y)
    R = 4.0 * rho * 0.6 ** 2 / 2.0
    Rr = 1.0 * 0.2
    np.testing.assert_allclose(f[:2], [-2 * R + 2 * Rr, R - Rr], rtol=1e-15)


def test_rhs_three_body_convention():
    """a + a + b -> c: rho^2 and 1/2!; a + b + d -> c (distinct): rho^2, no factorial."""
    from oracle import oracle as O
    spec = synth.NetworkSpec("three", np.array([1, 1, 3, 3]),
                             np.array([[0, 0, 1], [0, 1, 1]]), np.array([[2, -1, -1], [3, -1, -1]]),
                             np.array([[0.0] * 7, [math.log(5.0)] + [0.0] * 6]), np.zeros(2), 1.0)
    net = O.OracleNet(spec)
    y = np.array([0.3, 0.5, 0.0, 0.0, 1.0])
    rho = 3.0
    f = O.rhs(net, rho, y)
    R0 = 1.0 * rho ** 2 * 0.3 ** 2 * 0.5 / 2.0
    R1 = 5.0 * rho ** 2 * 0.3 * 0.5 ** 2 / 2.0
    np.testing.assert_allclose(f[:4], [-2 * R0 - R1, -R0 - 2 * R1, R0, R1], rtol=1e-15)


def test_rhs_robertson_hand_derived(oracle):
    """The config-1 network written out by hand at constant temperature:
    f_A = -k1 A + k3 B C + k4 C, f_B = k1 A - k2 rho B^2/2 - k3 rho B C,
    f_C = k2 rho B^2/2 - k4 C, f_T = (q1 k1 A + q2 k2 rho B^2/2 + q3 k3 rho B C + q4 k4 C)/c_v."""
    spec = synth.robertson_network()
    net = oracle.OracleNet(spec)
    T, rho = 2.2, 13.0
    lam, _ = oracle.rates(net, T)
    k1, k2, k3, k4 = lam
    A, B, Cc = 0.7, 2e-5, 0.29
    f = oracle.rhs(net, rho, [A, B, Cc, T])
    r2 = k2 * rho * B * B / 2
    r3 = k3 * rho * B * Cc
    exp = [-k1 * A + r3 + k4 * Cc, k1 * A - r2 - r3, r2 - k4 * Cc,
           (spec.q[0] * k1 * A + spec.q[1] * r2 + spec.q[2] * r3 + spec.q[3] * k4 * Cc) / spec.c_v]
    np.testing.assert_allclose(f, exp, rtol=1e-13)


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_rhs_mass_conservation(oracle, cfg):
    """sum_i A_i f_i = 0 for every state (every reaction conserves mass number)."""
    spec = synth.config(cfg, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(0)
    for _ in range(20):
        y = np.concatenate([rng.uniform(0, 1, spec.n_species), [rng.uniform(1, 5)]])
        f = oracle.rhs(net, 10 ** rng.uniform(0, 3), y)
        mag = np.abs(spec.mass * f[:-1]).sum()
        assert abs(np.dot(spec.mass, f[:-1])) <= 1e-14 * mag + 1e-300


def test_rhs_heat_identity(oracle):
    """One reaction with q: f_T c_v equals q times the product's rate."""
    spec = synth.chain_network([3.0], q=[2.5], c_v=4.0)
    net = oracle.OracleNet(spec)
    f = oracle.rhs(net, 1.0, [0.8, 0.2, 1.0])
    assert f[2] * 4.0 == pytest.approx(2.5 * f[1], rel=1e-15)


# ---------------------------------------------------------------------------
# Jacobian
# ---------------------------------------------------------------------------

def _fd_jac(oracle, net, rho, y):
    n = len(y)
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(1e-3, abs(y[j]))
        ys = []
        for m in (-2, -1, 1, 2):
            yy = np.array(y, dtype=np.float64)
            yy[j] += m * h
            ys.append(oracle.rhs(net, rho, yy))
        J[:, j] = (ys[0] - 8 * ys[1] + 8 * ys[2] - ys[3]) / (12 * h)
    return J


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_jacobian_vs_finite_differences(oracle, cfg):
    spec = synth.config(cfg, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(cfg)
    for _ in range(4):
        y = np.concatenate([rng.uniform(0.01, 1, spec.n_species), [rng.uniform(1.2, 4.5)]])
        rho = 10 ** rng.uniform(0, 2)
        J = oracle.jac(net, rho, y)
        Jfd = _fd_jac(oracle, net, rho, y)
        scale = np.abs(J).max()
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-8 * scale)


def _mp_rhs(spec, rho, y):
    """The right-hand side written from its definition (the rate law of the
    burn) in mpmath arithmetic; y may be complex (complex-step)."""
    N, R = spec.n_species, spec.n_reactions
    T = y[N]
    t13 = mpmath.cbrt(T)
    basis = [1, 1 / T, 1 / t13, t13, T, T * t13 * t13, mpmath.log(T)]
    f = [mpmath.mpf(0)] * (N + 1)
    for r in range(R):
        lam = mpmath.exp(sum(mpmath.mpf(float(spec.coef[r, k])) * basis[k] for k in range(7)))
        reac = [int(x) for x in spec.reactants[r] if x >= 0]
        rate = lam * mpmath.mpf(float(rho)) ** (len(reac) - 1)
        for sp in reac:
            rate *= y[sp]
        for sp in set(reac):
            rate /= math.factorial(reac.count(sp))
        for sp in reac:
            f[sp] -= rate
        for sp in spec.products[r]:
            if sp >= 0:
                f[int(sp)] += rate
        f[N] += mpmath.mpf(float(spec.q[r])) * rate / mpmath.mpf(float(spec.c_v))
    return f


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_jacobian_vs_complex_step(oracle, cfg):
    """The analytic Jacobian against the complex-step derivative of the rate
    law evaluated in 40-digit arithmetic (step 1e-30: exact to ~1e-60), entry
    by entry to 1e-13 of the entry's exact value."""
    spec = synth.config(cfg, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(100 + cfg)
    n = spec.n
    mpmath.mp.dps = 40
    try:
        for _ in range(2):
            y = np.concatenate([rng.uniform(0.01, 1, spec.n_species), [rng.uniform(1.2, 4.5)]])
            rho = 10 ** rng.uniform(0, 2)
            J = oracle.jac(net, rho, y)
            Jref = np.zeros((n, n))
            for j in range(n):
                yc = [mpmath.mpc(float(v)) for v in y]
                yc[j] += mpmath.mpc(0, 1e-30)
                fc = _mp_rhs(spec, rho, yc)
                Jref[:, j] = [float(mpmath.im(v) / mpmath.mpf("1e-30")) for v in fc]
            # each entry against its own exact value (a structural zero must
            # come out as exactly zero)
            rel = np.abs(J - Jref) / (np.abs(Jref) + 1e-300)
            print(f"config {cfg}: max relative entry error {rel.max():.2e}")
            assert rel.max() <= 1e-13, rel.max()
    finally:
        mpmath.mp.dps = 50


def test_jacobian_zero_abundance_and_structure(oracle):
    """With Y_j = 0 the slot-product derivative is still right (2B->B+C at B=0
    has dR/dB = 0 but B+C->A+C has dR/dB = k rho C); zero pattern matches the
    reactions."""
    spec = synth.robertson_network()
    net = oracle.OracleNet(spec)
    lam, _ = oracle.rates(net, 2.0)
    y = np.array([1.0, 0.0, 0.5, 2.0])
    J = oracle.jac(net, 3.0, y)
    # d f_B / d B = -k2 rho B - k3 rho C = -k3 rho C at B = 0
    assert J[1, 1] == pytest.approx(-lam[2] * 3.0 * 0.5, rel=1e-14)
    # A does not depend on ... f_C does not depend on A
    assert J[2, 0] == 0.0


@pytest.mark.parametrize("cfg", [2, 5])
def test_jacobian_mass_left_null_vector(oracle, cfg):
    """w^T J = 0 for w = (A, 0): differentiating sum_i A_i f_i = 0."""
    spec = synth.config(cfg, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    rng = np.random.default_rng(7)
    y = np.concatenate([rng.uniform(0, 1, spec.n_species), [3.3]])
    J = oracle.jac(net, 50.0, y)
    w = np.concatenate([spec.mass, [0]]).astype(float)
    lhs = w @ J
    mag = (np.abs(w)[:, None] * np.abs(J)).sum(0)
    assert np.all(np.abs(lhs) <= 1e-13 * mag + 1e-300)


# ---------------------------------------------------------------------------
# LU
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4, 14, 22, 51])
def test_lu_vs_lapack(oracle, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    LU, piv, info = oracle.lu_factor(A)
    assert info == 0
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(LU, lu_ref, rtol=1e-11, atol=1e-13)
    b = rng.standard_normal(n)
    x = oracle.lu_solve(LU, piv, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # backward error
    r = A @ x - b
    assert np.linalg.norm(r) <= 50 * n * np.finfo(float).eps * np.linalg.norm(A) * np.linalg.norm(x)


def test_lu_ties_go_to_lowest_row(oracle):
    A = np.array([[1.0, 2.0, 0.0], [-3.0, 1.0, 1.0], [3.0, 0.0, 2.0]])
    _, piv, info = oracle.lu_factor(A)
    assert info == 0 and piv[0] == 1  # |-3| == |3|: the first of the tied rows
    _, piv_ref = scipy.linalg.lu_factor(A)
    np.testing.assert_array_equal(piv, piv_ref)


def test_lu_singular_reported(oracle):
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 0.0, 1.0]])
    _, _, info = oracle.lu_factor(A)
    assert info == 2  # column 1 has no nonzero pivot


def test_lu_newton_matrix_of_network(oracle):
    """The Newton matrix I - cJ of a config-2 state: factor/solve residual."""
    spec = synth.config(2, n_cells=4).networks[0]
    net = oracle.OracleNet(spec)
    y = np.concatenate([np.full(spec.n_species, 0.05), [2.0]])
    J = oracle.jac(net, 100.0, y)
    M = np.eye(spec.n) - 1e-3 * J
    LU, piv, info = oracle.lu_factor(M)
    assert info == 0
    b = np.arange(1.0, spec.n + 1)
    x = oracle.lu_solve(LU, piv, b)
    np.testing.assert_allclose(M @ x, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


# ---------------------------------------------------------------------------
# Step-size change of the backward differences
# ---------------------------------------------------------------------------

def _backward_differences(values):
    """values[m] = p(t_n - m h): returns nabla^j p at t_n for j = 0..k."""
    k = len(values) - 1
    out = []
    for j in range(k + 1):
        out.append(sum(((-1) ** m) * math.comb(j, m) * values[m] for m in range(j + 1)))
    return np.array(out)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("rho_h", [0.2, 0.5, 0.9, 1.7, 10.0])
def test_rescale_reproduces_polynomial(oracle, k, rho_h):
    """Backward differences of a degree-k polynomial at step h, rescaled to
    step rho_h*h, equal the differences of the same polynomial taken at the
    new nodes (computed here directly from the polynomial)."""
    rng = np.random.default_rng(k)
    coeffs = rng.standard_normal((k + 1, 3))  # 3 components
    h = 0.3

    def p(t):
        return sum(coeffs[j] * t ** j for j in range(k + 1))

    old = _backward_differences([p(-m * h) for m in range(k + 1)])
    new_ref = _backward_differences([p(-m * rho_h * h) for m in range(k + 1)])
    new = oracle.rescale(old, k, rho_h)
    np.testing.assert_allclose(new, new_ref, rtol=1e-11, atol=1e-11 * np.abs(new_ref).max())


def test_rescale_identity_and_composition(oracle):
    rng = np.random.default_rng(3)
    D = rng.standard_normal((6, 4))
    np.testing.assert_allclose(oracle.rescale(D, 5, 1.0), D, rtol=1e-13, atol=1e-13)
    a = oracle.rescale(oracle.rescale(D, 4, 0.5), 4, 0.6)
    b = oracle.rescale(D, 4, 0.3)
    np.testing.assert_allclose(a[:5], b[:5], rtol=1e-11, atol=1e-11)
    np.testing.assert_array_equal(a[5], D[5])  # rows above k untouched
