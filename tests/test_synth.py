"""The seeded input generator: determinism and the construction rules the
workloads rely on (mass conservation, no cycles, every species used, rate
window)."""
import math

import mpmath
import numpy as np
import pytest

from paper_2312_02836_amd import synth


def _nu(net, r):
    v = {}
    for s in net.reactants[r]:
        if s >= 0:
            v[int(s)] = v.get(int(s), 0) - 1
    for s in net.products[r]:
        if s >= 0:
            v[int(s)] = v.get(int(s), 0) + 1
    return v


@pytest.mark.parametrize("ns,nr,seed", [(13, 30, 22), (21, 60, 55), (35, 100, 64), (50, 150, 33)])
def test_generator_rules(ns, nr, seed):
    net = synth.random_network(seed, ns, nr)
    net.validate()
    assert net.n_species == ns and net.n_reactions == nr
    phi = synth._potentials(net.mass)
    touched = set()
    keys = set()
    for r in range(nr):
        rs = tuple(int(s) for s in net.reactants[r] if s >= 0)
        ps = tuple(int(s) for s in net.products[r] if s >= 0)
        touched.update(rs + ps)
        # mass number conserved
        assert sum(net.mass[list(rs)]) == sum(net.mass[list(ps)])
        # strictly raises the potential -> no cycles
        assert phi[list(ps)].sum() > phi[list(rs)].sum()
        keys.add((rs, ps))
        assert any(_nu(net, r).values())
    assert len(keys) == nr, "duplicate reaction"
    assert touched == set(range(ns))
    # heat and c_v
    assert np.all((net.q >= 0) & (net.q <= 5)) and net.c_v == 100.0


def test_generator_rate_window():
    """Every rate of the config-2 network lies in [1e-6, 1e8] for T in [1, 5]
    (evaluated here with mpmath, independently of the generator's bound)."""
    net = synth.config(2, n_cells=4).networks[0]
    for r in range(net.n_reactions):
        a = [mpmath.mpf(float(x)) for x in net.coef[r]]
        for T in np.linspace(1.0, 5.0, 33):
            T = mpmath.mpf(float(T))
            lam = mpmath.exp(a[0] + a[1] / T + a[2] * T ** (-mpmath.mpf(1) / 3) + a[3] * mpmath.cbrt(T)
                             + a[4] * T + a[5] * T ** (mpmath.mpf(5) / 3) + a[6] * mpmath.log(T))
            assert 1e-6 <= lam <= 1e8


def test_generator_deterministic():
    a = synth.config(2, n_cells=64)
    b = synth.config(2, n_cells=64)
    assert a.networks[0].to_json() == b.networks[0].to_json()
    np.testing.assert_array_equal(a.cells[0].Y, b.cells[0].Y)
    np.testing.assert_array_equal(a.cells[0].T, b.cells[0].T)
    c = synth.random_network(23, 13, 30)
    assert c.to_json() != a.networks[0].to_json()


def test_cells_distributions():
    cfg = synth.config(2, n_cells=4096)
    c = cfg.cells[0]
    assert c.Y.shape == (13, 4096)
    seeds = synth.seed_species(cfg.networks[0])
    np.testing.assert_allclose(c.Y[seeds].sum(0), 1.0, rtol=0, atol=1e-15)
    others = np.setdiff1d(np.arange(13), seeds)
    assert np.all(c.Y[others] == 0)
    assert c.T.min() >= 1.0 and c.T.max() <= 5.0
    assert c.rho.min() >= 1.0 and c.rho.max() <= 1e3
    # log-uniform density: mean of log10 rho near 1.5
    assert abs(np.log10(c.rho).mean() - 1.5) < 0.05


def test_robertson_network():
    net = synth.robertson_network()
    assert net.describe() == ["s0 -> s1", "s1 + s1 -> s1 + s2", "s1 + s2 -> s0 + s2", "s2 -> s0"]
    targets = [1e-2, 1e7, 1e4, 1e-3]
    np.testing.assert_allclose(np.exp(net.coef[:, 0]), targets, rtol=1e-12)


def test_network_json_roundtrip_and_validation():
    net = synth.config(2, n_cells=4).networks[0]
    back = synth.NetworkSpec.from_json(net.to_json())
    assert back.to_json() == net.to_json()
    bad = synth.NetworkSpec.from_json(net.to_json())
    bad.products[0, 0] = (bad.products[0, 0] + 1) % bad.n_species
    with pytest.raises(ValueError):
        # one reaction's products changed -> mass number not conserved (all
        # species in this network have distinct neighbours' masses)
        for _ in range(bad.n_species):
            bad.validate()
            bad.products[0, 0] = (bad.products[0, 0] + 1) % bad.n_species


@pytest.mark.parametrize("i", [2, 3, 4, 5])
def test_networks_react_from_seed_composition(i):
    """Every workload network has at least three reactions whose reactants
    are all seed species, so a burn from the seed composition is not inert."""
    cfg = synth.config(i, n_cells=4)
    for net in cfg.networks:
        seeds = set(synth.seed_species(net).tolist())
        k = sum(all(s in seeds for s in net.reactants[r] if s >= 0)
                for r in range(net.n_reactions))
        assert k >= 3, (net.name, k)


def test_synth50_t_end_is_the_calibrated_value():
    """The 50/150 workload's burn time is the one the committed calibration
    (the oracle's step-count spread on 4,096 cells) chose."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "synth50_t_end.txt")
    with open(path) as f:
        val = [float(l.split("=")[1]) for l in f if l.startswith("t_end =")][0]
    assert synth.config(3, n_cells=8).t_end == val == synth.SYNTH50_T_END
