"""The parity gate itself (host logic): what it accepts and what it rejects."""
import numpy as np
import pytest

from tests.parity import ROUNDING_SENSITIVE_MIN_COUNTER_EQUAL, assert_parity

RT, AT = 1e-6, 1e-10


def _case(n_cells=200, seed=0):
    rng = np.random.default_rng(seed)
    Y = rng.uniform(0.1, 1.0, size=(3, n_cells))
    T = rng.uniform(1.0, 2.0, size=n_cells)
    st = np.zeros(n_cells, dtype=np.int32)
    cnt = rng.integers(1, 100, size=(8, n_cells)).astype(np.int32)
    return Y, T, st, cnt


def _copy(c):
    return tuple(np.array(x, copy=True) for x in c)


def test_identical_passes():
    o = _case()
    assert_parity(_copy(o), o, RT, AT)


def test_same_counters_beyond_tolerance_fails():
    o = _case()
    g = _copy(o)
    g[0][1, 7] *= 1.0 + 3 * RT
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT)


def test_status_mismatch_fails():
    o = _case()
    g = _copy(o)
    g[2][3] = 1
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT)


def test_divergent_cell_checked_against_tight_reference():
    o = _case()
    g = _copy(o)
    g[3][0, 11] += 1                  # a different decision sequence
    g[0][2, 11] *= 1.0 + 5 * RT       # 5x the tolerance away from the oracle
    m = ROUNDING_SENSITIVE_MIN_COUNTER_EQUAL
    # no tight reference: rejected
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT, min_counter_equal=m)
    # the tight solution sits near the GPU result: accepted
    assert_parity(g, o, RT, AT, min_counter_equal=m,
                  tight=lambda idx: (g[0][:, idx], g[1][idx]))
    # the tight solution is far (300 tolerances) from the GPU result: rejected
    far = lambda idx: (g[0][:, idx] * (1.0 + 300 * RT), g[1][idx])  # noqa: E731
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT, min_counter_equal=m, tight=far)


def test_default_gate_allows_no_divergence_in_small_samples():
    """The default share (99.9 %) leaves no divergent cell in a sample of
    fewer than 1000 cells, even one that is within the tolerance."""
    o = _case()
    g = _copy(o)
    g[3][0, 11] += 1
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT)


def test_too_many_divergent_cells_fail():
    o = _case()
    g = _copy(o)
    g[3][0, :10] += 1                 # 5 % of the cells
    with pytest.raises(AssertionError):
        assert_parity(g, o, RT, AT)
    assert_parity(g, o, RT, AT, min_counter_equal=0.9)
