"""Algorithmic FP64 operation counts of a burn, from the per-cell counters.

Every operation the method must perform is counted once: add, mul, fma (2),
division, square root and each transcendental (exp, log, cbrt, pow) as one
operation, whatever its cost in instructions on a given chip.

Two models.  ``path_cell_flops`` is the one the roofline fraction uses: per
right-hand side, Jacobian, Newton matrix and LU, solve and step attempt, the
operations of the method's definition (n = N + 1; per reaction r: m_r
reactant slots, u_r distinct reactant species, s_r species with nu != 0):

  F_rhs   = c_T + sum_r (15 + m_r + 2 s_r)      c_T = log + cbrt + div + 4 mul
  F_jac   = c_T + sum_r (25 + 2 u_r + 2 s_r (u_r + 1) + 2 (u_r + 1))
  F_M     = n^2 + n                              I - cJ
  F_LU    = n(n-1)/2 + n(n-1)(2n-1)/3
  F_solve = 2 n^2 - n  (+ 6 n of Newton vector work per solve)
  F_step  = (3 k + 10) n per step attempt        (k: the cell's final order)

  F_cell = n_rhs F_rhs + n_jac F_jac + n_lu (F_M + F_LU)
           + n_solve (F_solve + 6 n) + (n_steps + n_rej + n_fail) F_step

``cell_flops`` is a heavier accounting of the same burn (it also counts the
history update, the rescale and the order-choice norms), reported beside it:

  F_rhs    T powers (6) + per reaction r: exponent (12) + exp + multiplier +
           1/prod(m!) + rho^(n_r-1) + the n_r abundance factors + heat (2),
           + 2 per nonzero stoichiometric entry + 1 for the temperature row
  F_jac    rates with d ln(lambda)/dT, the slot-product derivatives of every
           (row, reaction) pair and the temperature row
  F_lu     I - cJ (2 n^2) + partial-pivot LU: n reciprocals + n(n-1)/2
           multipliers + n(n-1)(2n-1)/3 for the trailing updates
  F_solve  forward + back substitution (2 n^2 - n) + the Newton vector work
           (8 n + 3: right side, weighted norm, updates)
  F_att    per step attempt: predictor, psi, scales and error test at the
           highest order ((3*5 + 13) n)
  F_acc    per accepted step: history update and order-choice norms (14 n)
  F_resc   per step-size change: the (k+1)^2 history transform at k = 5
           (132 n); the number of changes is estimated as n_lu - n_jac

F_cell = n_rhs F_rhs + n_jac F_jac + n_lu F_lu + n_solve F_solve
         + (n_steps + n_rej + n_fail) F_att + n_steps F_acc + n_resc F_resc
"""
from __future__ import annotations

import numpy as np


def _reaction_shape(spec):
    """Per reaction: reactant slots m_r, distinct reactant species u_r, and
    species with a nonzero net coefficient s_r."""
    m, u, s = [], [], []
    for r in range(spec.n_reactions):
        reac = [int(x) for x in spec.reactants[r] if x >= 0]
        nu = {}
        for x in reac:
            nu[x] = nu.get(x, 0) - 1
        for x in spec.products[r]:
            if x >= 0:
                nu[int(x)] = nu.get(int(x), 0) + 1
        m.append(len(reac))
        u.append(len(set(reac)))
        s.append(sum(1 for v in nu.values() if v))
    return np.array(m, np.int64), np.array(u, np.int64), np.array(s, np.int64)


def path_costs(spec) -> dict:
    """Operations per evaluation in the hot-path model (module docstring)."""
    n = spec.n
    m, u, s = _reaction_shape(spec)
    c_t = 7
    return {"rhs": c_t + int((15 + m + 2 * s).sum()),
            "jac": c_t + int((25 + 2 * u + 2 * s * (u + 1) + 2 * (u + 1)).sum()),
            "m": n * n + n,
            "lu": n * (n - 1) // 2 + n * (n - 1) * (2 * n - 1) // 3,
            "solve": 2 * n * n - n + 6 * n}


def path_cell_flops(spec, counters: np.ndarray) -> np.ndarray:
    """Per-cell operation count of the hot-path model; counters is [8, C]."""
    c = np.asarray(counters, dtype=np.int64)
    n_steps, n_rej, n_fail, n_rhs, n_jac, n_lu, n_solve, order = c[:8]
    k = path_costs(spec)
    n = spec.n
    return (n_rhs * k["rhs"] + n_jac * k["jac"] + n_lu * (k["m"] + k["lu"])
            + n_solve * k["solve"] + (n_steps + n_rej + n_fail) * (3 * order + 10) * n)


def path_total_flops(spec, counters: np.ndarray) -> float:
    return float(path_cell_flops(spec, counters).sum())


def per_eval_costs(spec) -> dict:
    n = spec.n
    nr = (spec.reactants >= 0).sum(axis=1).astype(np.int64)
    nu_nz = []
    for r in range(spec.n_reactions):
        v = {}
        for s in spec.reactants[r]:
            if s >= 0:
                v[int(s)] = v.get(int(s), 0) - 1
        for s in spec.products[r]:
            if s >= 0:
                v[int(s)] = v.get(int(s), 0) + 1
        nu_nz.append(sum(1 for x in v.values() if x))
    nu_nz = np.array(nu_nz, dtype=np.int64)
    nnz = int(nu_nz.sum())
    f_rhs = 7 + int((17 + 2 * nr).sum()) + 2 * nnz
    f_jac = 6 + int((34 + 2 * nr).sum()) + int((nu_nz * (nr * (nr + 1) + 2)).sum()) + int(
        (nr * (nr + 2) + 3).sum())
    f_lu = 2 * n * n + n + n * (n - 1) // 2 + n * (n - 1) * (2 * n - 1) // 3
    f_solve = 2 * n * n - n + 8 * n + 3
    return {"rhs": f_rhs, "jac": f_jac, "lu": f_lu, "solve": f_solve, "att": 28 * n,
            "acc": 14 * n, "resc": 132 * n}


def cell_flops(spec, counters: np.ndarray) -> np.ndarray:
    """Per-cell algorithmic operation count; counters is [8, C]."""
    c = np.asarray(counters, dtype=np.int64)
    n_steps, n_rej, n_fail, n_rhs, n_jac, n_lu, n_solve = c[:7]
    k = per_eval_costs(spec)
    n_resc = np.maximum(n_lu - n_jac, 0)
    return (n_rhs * k["rhs"] + n_jac * k["jac"] + n_lu * k["lu"] + n_solve * k["solve"]
            + (n_steps + n_rej + n_fail) * k["att"] + n_steps * k["acc"] + n_resc * k["resc"])


def total_flops(spec, counters: np.ndarray) -> float:
    return float(cell_flops(spec, counters).sum())


def adjoint_cell_flops(spec, counters: np.ndarray, replay_iters: np.ndarray,
                       recomputed=False) -> np.ndarray:
    """Per-cell algorithmic operation count of one sensitivity run (recording
    burn, replay with exact correctors and the reverse sweep), from the
    recording run's counters [8, C] and the replay's Newton iterations and
    factorizations [2, C].  recomputed (bool, or per cell) adds the second
    replay of a cell whose corrected states were recomputed from checkpoints
    for the reverse sweep (the cells the state pool did not hold).

      recording     cell_flops (the production burn)
      replay        iterations x (F_rhs + F_solve) + factorizations x
                    (F_jac + F_lu), plus per accepted step the rescale,
                    predictor and update (174 n)
      reverse       per accepted step: Newton matrix and factors at the
                    corrected state (F_jac + F_lu), the transposed solve
                    (2 n^2 - n), the per-reaction contraction with J^T and
                    the gradient (F_jac + 2 nnz), and the transposed linear
                    history maps (60 n)
    """
    c = np.asarray(counters, dtype=np.int64)
    ri = np.asarray(replay_iters, dtype=np.int64)
    it, nf = ri[0], ri[1]
    n_steps = c[0]
    k = per_eval_costs(spec)
    n = spec.n
    reps = 1 + np.asarray(recomputed, dtype=np.int64)
    f_replay = it * (k["rhs"] + k["solve"]) + nf * (k["jac"] + k["lu"]) + n_steps * 174 * n
    f_rev = 2 * k["jac"] + k["lu"] + (2 * n * n - n) + 60 * n + 2 * spec.n_reactions * 6
    return (cell_flops(spec, counters) + reps * f_replay + n_steps * f_rev
            + k["rhs"] + k["jac"])
