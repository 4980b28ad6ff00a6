"""Seeded synthetic inputs for the per-cell reaction burn.

The paper's networks are built from the JINA ReacLib collection and tabulated
weak rates (paper, Sec. 2, "Arbitrary Network Generation").  Neither data set
is used here: every network is a seeded synthetic mass-action network whose
rate coefficients have the ReacLib seven-parameter form, and every batch of
cells is drawn from seeded distributions.

This module only draws numbers.  It evaluates no rate, right-hand side,
Jacobian or integrator step, so both the plain CPU oracle and the GPU path can
take their inputs from it without sharing any of the method's arithmetic.
The one place where the rate's temperature basis enters is the placement of
the constant coefficient a0 (``_place_a0``), which uses only the sup-norm of
each basis function on the temperature window, i.e. fixed constants.

A network is a :class:`NetworkSpec`; a batch of cells is a :class:`Cells`
with structure-of-arrays layout (``Y[N][C]``: species-major, so consecutive
cells are consecutive in memory).
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Number of fit coefficients in the ReacLib rate form a0..a6.
N_COEF = 7
# Reactant / product slots per reaction; unused slots hold -1.
N_SLOTS = 3


@dataclasses.dataclass
class NetworkSpec:
    """A mass-action reaction network (host arrays, plain numpy).

    mass       int32[N]       mass number A_i >= 1 of each species
    reactants  int32[R, 3]    species index per reactant slot, -1 pad;
                              a repeated index is a multiplicity (2B -> (B,B,-1))
    products   int32[R, 3]    same convention for products
    coef       float64[R, 7]  ReacLib-form coefficients a0..a6
    q          float64[R]     heat released per reaction event
    c_v        float          constant specific heat (> 0)
    screen     float64[R] or None  strengths h_r of the synthetic screening
                              factor exp(h_r G(rho, T, Y)) (None: no screening)
    """

    name: str
    mass: np.ndarray
    reactants: np.ndarray
    products: np.ndarray
    coef: np.ndarray
    q: np.ndarray
    c_v: float
    screen: Optional[np.ndarray] = None

    @property
    def n_species(self) -> int:
        return int(self.mass.shape[0])

    @property
    def n_reactions(self) -> int:
        return int(self.reactants.shape[0])

    @property
    def n(self) -> int:
        """Size of the ODE system: species plus temperature."""
        return self.n_species + 1

    def __post_init__(self):
        self.mass = np.ascontiguousarray(self.mass, dtype=np.int32)
        self.reactants = np.ascontiguousarray(self.reactants, dtype=np.int32).reshape(-1, N_SLOTS)
        self.products = np.ascontiguousarray(self.products, dtype=np.int32).reshape(-1, N_SLOTS)
        self.coef = np.ascontiguousarray(self.coef, dtype=np.float64).reshape(-1, N_COEF)
        self.q = np.ascontiguousarray(self.q, dtype=np.float64).reshape(-1)
        self.c_v = float(self.c_v)
        if self.screen is not None:
            self.screen = np.ascontiguousarray(self.screen, dtype=np.float64).reshape(-1)

    def validate(self) -> None:
        """Raise ValueError unless indices are in range and every reaction
        conserves mass number (sum of A over reactant slots equals the sum
        over product slots)."""
        N, R = self.n_species, self.n_reactions
        if N < 1 or R < 1:
            raise ValueError("network needs at least one species and one reaction")
        if np.any(self.mass < 1):
            raise ValueError("mass numbers must be >= 1")
        for arr, what in ((self.reactants, "reactant"), (self.products, "product")):
            if np.any((arr < -1) | (arr >= N)):
                raise ValueError(f"{what} index out of range")
        if self.coef.shape != (R, N_COEF) or self.q.shape != (R,):
            raise ValueError("coef must be [R,7] and q must be [R]")
        if not (self.c_v > 0 and math.isfinite(self.c_v)):
            raise ValueError("c_v must be positive and finite")
        if self.screen is not None and (self.screen.shape != (R,)
                                        or not np.all(np.isfinite(self.screen))):
            raise ValueError("screen must be [R] and finite")
        for r in range(R):
            rs = [int(s) for s in self.reactants[r] if s >= 0]
            ps = [int(s) for s in self.products[r] if s >= 0]
            if not rs:
                raise ValueError(f"reaction {r} has no reactant")
            if sum(int(self.mass[s]) for s in rs) != sum(int(self.mass[s]) for s in ps):
                raise ValueError(f"reaction {r} does not conserve mass number")

    def to_json(self) -> str:
        return json.dumps({
            "name": self.name, "mass": self.mass.tolist(),
            "reactants": self.reactants.tolist(), "products": self.products.tolist(),
            "coef": self.coef.tolist(), "q": self.q.tolist(), "c_v": self.c_v,
            "screen": None if self.screen is None else self.screen.tolist()})

    @staticmethod
    def from_json(text: str) -> "NetworkSpec":
        d = json.loads(text)
        return NetworkSpec(d["name"], np.array(d["mass"]), np.array(d["reactants"]),
                           np.array(d["products"]), np.array(d["coef"]), np.array(d["q"]),
                           d["c_v"], None if d.get("screen") is None else np.array(d["screen"]))

    def describe(self) -> List[str]:
        """Human-readable reaction list, e.g. ``s0 + s1 -> s2``."""
        out = []
        for r in range(self.n_reactions):
            lhs = " + ".join(f"s{s}" for s in self.reactants[r] if s >= 0)
            rhs = " + ".join(f"s{s}" for s in self.products[r] if s >= 0) or "(nothing)"
            out.append(f"{lhs} -> {rhs}")
        return out


@dataclasses.dataclass
class Cells:
    """A batch of independent cells, structure-of-arrays.

    Y    float64[N, C]  initial molar abundances
    rho  float64[C]     density (constant during the burn)
    T    float64[C]     initial temperature
    """

    Y: np.ndarray
    rho: np.ndarray
    T: np.ndarray

    @property
    def n_cells(self) -> int:
        return int(self.rho.shape[0])

    def subset(self, idx: np.ndarray) -> "Cells":
        idx = np.asarray(idx)
        return Cells(np.ascontiguousarray(self.Y[:, idx]), np.ascontiguousarray(self.rho[idx]),
                     np.ascontiguousarray(self.T[idx]))


@dataclasses.dataclass
class BurnConfig:
    """One benchmark/test configuration: network(s), cells and integration knobs."""

    name: str
    networks: List[NetworkSpec]
    cells: List[Cells]
    t_end: float
    rtol: float = 1e-6
    atol: float = 1e-10


# ---------------------------------------------------------------------------
# Coefficient draws
# ---------------------------------------------------------------------------

# Half-widths of the uniform draws for a1..a6 (a1 larger, a5 much smaller
# because T^(5/3) grows fastest on the window).
_A_HALF_WIDTH = np.array([2.0, 0.5, 0.5, 0.5, 0.05, 0.5])


def _basis_sup(t_lo: float, t_hi: float) -> np.ndarray:
    """Sup-norm of each temperature basis function (1/T, T^-1/3, T^1/3, T,
    T^5/3, ln T) on [t_lo, t_hi].  All six are monotone, so the sup-norm is the
    larger magnitude at the two end points."""
    def mags(t):
        return np.array([1.0 / t, t ** (-1.0 / 3.0), t ** (1.0 / 3.0), t, t ** (5.0 / 3.0),
                         abs(math.log(t))])
    return np.maximum(mags(t_lo), mags(t_hi))


def _draw_shape(rng: np.random.Generator, n: int) -> np.ndarray:
    """a1..a6 for n reactions, uniform in +-half-width."""
    return rng.uniform(-1.0, 1.0, size=(n, 6)) * _A_HALF_WIDTH


def _place_a0(rng: np.random.Generator, shape: np.ndarray, t_window: Tuple[float, float],
              lam_window: Tuple[float, float]) -> np.ndarray:
    """Draw a0 uniformly inside the window that keeps the rate within
    lam_window for every T in t_window, using the bound
    |sum_k a_k phi_k(T)| <= sum_k |a_k| sup|phi_k|."""
    sup = _basis_sup(*t_window)
    bound = np.abs(shape) @ sup
    lo = math.log(lam_window[0]) + bound
    hi = math.log(lam_window[1]) - bound
    if np.any(hi <= lo):
        raise ValueError("rate window too narrow for the drawn temperature dependence")
    return rng.uniform(lo, hi)


# ---------------------------------------------------------------------------
# Networks
# ---------------------------------------------------------------------------

ROBERTSON_SEED = 20231205


def robertson_network(seed: int = ROBERTSON_SEED, c_v: float = 100.0) -> NetworkSpec:
    """Three species (A, B, C; all mass number 1) and four reactions with a
    Robertson-like spread of time scales:

      A -> B          slow          (target rate 1e-2)
      B + B -> B + C  fast          (target rate 1e7)
      B + C -> A + C  intermediate  (target rate 1e4)
      C -> A          slowest       (target rate 1e-3), closing the cycle

    a0 = ln(target); a1..a6 are seeded small, so the rate at T in [1,3] sits
    within a few e-folds of its target.  q ~ U[0,5].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    targets = np.array([1e-2, 1e7, 1e4, 1e-3])
    shape = _draw_shape(rng, 4)
    coef = np.concatenate([np.log(targets)[:, None], shape], axis=1)
    reactants = np.array([[0, -1, -1], [1, 1, -1], [1, 2, -1], [2, -1, -1]])
    products = np.array([[1, -1, -1], [1, 2, -1], [0, 2, -1], [0, -1, -1]])
    q = rng.uniform(0.0, 5.0, size=4)
    net = NetworkSpec("robertson3", np.array([1, 1, 1]), reactants, products, coef, q, c_v)
    net.validate()
    return net


def _species_masses(rng: np.random.Generator, n_species: int) -> np.ndarray:
    """Integer mass numbers, sorted, with at least two light species so that
    captures exist, and isobars allowed."""
    max_mass = max(4, (3 * n_species) // 2)
    while True:
        m = np.sort(rng.integers(1, max_mass + 1, size=n_species))
        m[0] = 1
        m[1] = min(m[1], 2)
        m = np.sort(m)
        if len(set(m.tolist())) >= max(3, n_species // 2):
            return m.astype(np.int32)


def _potentials(mass: np.ndarray) -> np.ndarray:
    """Per-species potential Phi_s = A_s^2 + eps * (rank among isobars).
    Every generated reaction strictly raises the summed potential, so the
    network has no cycles and a bounded number of reaction events."""
    n = len(mass)
    rank = np.zeros(n)
    seen: Dict[int, int] = {}
    for i, a in enumerate(mass.tolist()):
        rank[i] = seen.get(a, 0)
        seen[a] = seen.get(a, 0) + 1
    eps = 0.25 / max(1, n)
    return mass.astype(np.float64) ** 2 + eps * rank


def _candidates(mass: np.ndarray) -> Dict[str, List[Tuple[Tuple[int, ...], Tuple[int, ...]]]]:
    """All mass-conserving candidate reactions that raise the potential,
    by kind: isobaric decays a->b, captures a+b->c, three-body captures
    a+b+d->c and exchanges a+b->c+d."""
    n = len(mass)
    phi = _potentials(mass)
    A = mass.tolist()
    out: Dict[str, list] = {"one": [], "capture": [], "exchange": [], "three": []}
    for a in range(n):
        for b in range(n):
            if a != b and A[a] == A[b] and phi[b] > phi[a]:
                out["one"].append(((a,), (b,)))
    for a in range(n):
        for b in range(a, n):
            for c in range(n):
                if A[c] == A[a] + A[b] and phi[c] > phi[a] + phi[b]:
                    out["capture"].append(((a, b), (c,)))
            for c in range(n):
                for d in range(c, n):
                    if (c, d) == (a, b):
                        continue
                    if A[c] + A[d] == A[a] + A[b] and phi[c] + phi[d] > phi[a] + phi[b] + 1e-12:
                        out["exchange"].append(((a, b), (c, d)))
            for d in range(b, n):
                for c in range(n):
                    if A[c] == A[a] + A[b] + A[d] and phi[c] > phi[a] + phi[b] + phi[d]:
                        out["three"].append(((a, b, d), (c,)))
    return out


def _touched(chosen) -> set:
    out = set()
    for rs, ps in chosen:
        out.update(rs)
        out.update(ps)
    return out


def _ensure_seed_reactions(rng, mass, chosen, pools, k_min):
    """Replace reactions until at least k_min have only seed reactants; None
    if that cannot be done while every species stays in some reaction."""
    seeds = set(np.argsort(_potentials(mass), kind="stable")[:3].tolist())

    def seed_only(rx):
        return all(s in seeds for s in rx[0])

    have = sum(seed_only(c) for c in chosen)
    if have >= k_min:
        return chosen
    n_species = len(mass)
    pool = [c for pl in pools for c in pl if seed_only(c) and c not in chosen]
    need = min(k_min - have, len(pool))
    if need <= 0:
        return chosen
    picks = sorted(rng.choice(len(pool), size=need, replace=False).tolist())
    chosen = list(chosen)
    for i in picks:
        new = pool[i]
        for idx in rng.permutation(len(chosen)).tolist():
            if seed_only(chosen[idx]):
                continue
            trial = chosen[:idx] + chosen[idx + 1:] + [new]
            if len(_touched(trial)) == n_species:
                chosen = trial
                break
        else:
            return None
    return chosen


def random_network(seed: int, n_species: int, n_reactions: int, *, name: Optional[str] = None,
                   mix: Tuple[float, float, float] = (0.20, 0.65, 0.15),
                   t_window: Tuple[float, float] = (1.0, 5.0),
                   lam_window: Tuple[float, float] = (1e-6, 1e8),
                   c_v: float = 100.0, min_seed_reactions: int = 3) -> NetworkSpec:
    """Seeded acyclic mass-action network with 1-, 2- and 3-body reactions.

    mix = fractions of (1-body, 2-body, 3-body) reactions; 2-body reactions
    are captures a+b->c and exchanges a+b->c+d.  Every reaction conserves mass
    number and raises the species potential (no cycles, bounded heating).
    Every species takes part in at least one reaction; no duplicates.
    At least min_seed_reactions reactions have only seed species (the three
    of lowest potential, which start the burn) as reactants, so that a burn
    from a seed composition is not trivially inert: a network drawn without
    enough of them has randomly chosen other reactions replaced by seed-only
    candidates (networks that already have enough are left as drawn).
    a1..a6 are drawn small and a0 is placed so every rate lies in lam_window
    over t_window.  q_r ~ U[0,5]; c_v constant.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    for _attempt in range(200):
        mass = _species_masses(rng, n_species)
        cand = _candidates(mass)
        two = cand["capture"] + cand["exchange"]
        want = [int(round(mix[0] * n_reactions)), 0, int(round(mix[2] * n_reactions))]
        want[1] = n_reactions - want[0] - want[2]
        pools = [cand["one"], two, cand["three"]]
        # Move any shortfall of a kind to the two-body pool.
        for k in (0, 2):
            if len(pools[k]) < want[k]:
                want[1] += want[k] - len(pools[k])
                want[k] = len(pools[k])
        if len(pools[1]) < want[1]:
            continue
        chosen: List[Tuple[Tuple[int, ...], Tuple[int, ...]]] = []
        for k in range(3):
            if want[k]:
                idx = rng.choice(len(pools[k]), size=want[k], replace=False)
                chosen += [pools[k][i] for i in sorted(idx)]
        if len(_touched(chosen)) != n_species:
            continue
        chosen = _ensure_seed_reactions(rng, mass, chosen, pools, min_seed_reactions)
        if chosen is None:
            continue
        break
    else:
        raise RuntimeError("could not draw a network that touches every species")

    R = n_reactions
    reactants = -np.ones((R, N_SLOTS), dtype=np.int32)
    products = -np.ones((R, N_SLOTS), dtype=np.int32)
    for r, (rs, ps) in enumerate(chosen):
        reactants[r, :len(rs)] = sorted(rs)
        products[r, :len(ps)] = sorted(ps)
    shape = _draw_shape(rng, R)
    a0 = _place_a0(rng, shape, t_window, lam_window)
    coef = np.concatenate([a0[:, None], shape], axis=1)
    q = rng.uniform(0.0, 5.0, size=R)
    net = NetworkSpec(name or f"synth{n_species}x{n_reactions}s{seed}", mass, reactants, products,
                      coef, q, c_v)
    net.validate()
    return net


def seed_species(net: NetworkSpec, k: int = 3) -> np.ndarray:
    """The k species of lowest potential (the lightest ones), which start the burn."""
    phi = _potentials(net.mass)
    return np.argsort(phi, kind="stable")[:k]


# ---------------------------------------------------------------------------
# Cells
# ---------------------------------------------------------------------------

def draw_cells(seed: int, net: NetworkSpec, n_cells: int, *,
               T_range: Tuple[float, float] = (1.0, 5.0), T_log: bool = False,
               rho_range: Tuple[float, float] = (1.0, 1e3),
               y0: Optional[Sequence[float]] = None, n_seed_species: int = 3) -> Cells:
    """Seeded cells: T uniform (or log-uniform) in T_range, rho log-uniform in
    rho_range, and Y0 either the given vector for every cell or
    Dirichlet(1,...,1) over the network's seed species (others zero)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if T_log:
        T = np.exp(rng.uniform(math.log(T_range[0]), math.log(T_range[1]), size=n_cells))
    else:
        T = rng.uniform(T_range[0], T_range[1], size=n_cells)
    rho = np.exp(rng.uniform(math.log(rho_range[0]), math.log(rho_range[1]), size=n_cells))
    N = net.n_species
    Y = np.zeros((N, n_cells))
    if y0 is not None:
        Y[:, :] = np.asarray(y0, dtype=np.float64)[:, None]
    else:
        seeds = seed_species(net, n_seed_species)
        Y[seeds, :] = rng.dirichlet(np.ones(len(seeds)), size=n_cells).T
    return Cells(np.ascontiguousarray(Y), np.ascontiguousarray(rho), np.ascontiguousarray(T))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

CONFIG_SEEDS = {1: 11, 2: 22, 3: 33, 4: 44, 5: 55}
MIXED_SIZES = [(13, 30), (21, 60), (35, 100), (50, 150)]

# Burn time of the 50/150 workload: chosen so that the 95th / 5th percentile
# ratio of the accepted-step counts is about 10 (10.7 on a 4,096-cell sample;
# tests/golden/calibrate_synth50_t_end.py, which calls the oracle, wrote the
# value to tests/golden/synth50_t_end.txt).
SYNTH50_T_END = 3e-4


def config(i: int, n_cells: Optional[int] = None) -> BurnConfig:
    """The synthetic workloads (sizes and distributions as described in the
    design notes).  ``n_cells`` overrides the cell count per network (the
    draws for the first n cells are the same for any larger count only when
    the generator is asked for that larger count; tests use the full draw and
    slice it)."""
    s = CONFIG_SEEDS[i]
    if i == 1:
        net = robertson_network()
        C = n_cells or 256
        cells = draw_cells(s, net, C, T_range=(1.0, 3.0), rho_range=(1.0, 1e2), y0=[1.0, 0.0, 0.0])
        return BurnConfig("robertson3-256", [net], [cells], t_end=1e3)
    if i == 2:
        net = random_network(s, 13, 30)
        C = n_cells or 65536
        cells = draw_cells(s + 1, net, C, T_range=(1.0, 5.0), rho_range=(1.0, 1e3))
        return BurnConfig("synth13x30-65536", [net], [cells], t_end=1e-2)
    if i == 3:
        net = random_network(s, 50, 150)
        C = n_cells or 1048576
        cells = draw_cells(s + 1, net, C, T_range=(0.8, 6.0), T_log=True, rho_range=(1.0, 1e3))
        return BurnConfig("synth50x150-1M", [net], [cells], t_end=SYNTH50_T_END)
    if i == 4:
        nets = [random_network(s + 10 * j, ns, nr) for j, (ns, nr) in enumerate(MIXED_SIZES)]
        C = n_cells or 65536
        cells = [draw_cells(s + 10 * j + 1, nt, C, T_range=(1.0, 5.0), rho_range=(1.0, 1e3))
                 for j, nt in enumerate(nets)]
        return BurnConfig("mixed4-4x65536", nets, cells, t_end=1e-2)
    if i == 5:
        net = random_network(s, 21, 60)
        C = n_cells or 65536
        cells = draw_cells(s + 1, net, C, T_range=(1.0, 5.0), rho_range=(1.0, 1e3))
        return BurnConfig("adjoint21x60-65536", [net], [cells], t_end=1e-2)
    raise KeyError(i)


def screened(net: NetworkSpec, strength: float = 0.005) -> NetworkSpec:
    """The same network with synthetic screening: h_r = strength times
    (number of reactants - 1), so one-body reactions are unscreened and
    three-body ones twice as strongly as two-body ones.  With rho <= 1e3 and
    T >= 1, G <= ~300 on the workloads, so h_r G stays O(1).  (A stand-in for
    real screening; no plasma data is used.)"""
    h = np.zeros(net.n_reactions)
    for r in range(net.n_reactions):
        k = int((net.reactants[r] >= 0).sum())
        h[r] = strength * (k - 1)
    return NetworkSpec(net.name + "-screened", net.mass.copy(), net.reactants.copy(),
                       net.products.copy(), net.coef.copy(), net.q.copy(), net.c_v, h)


# ---------------------------------------------------------------------------
# Small textbook networks used by the tests
# ---------------------------------------------------------------------------

def chain_network(rates: Sequence[float], q: Optional[Sequence[float]] = None,
                  c_v: float = 100.0) -> NetworkSpec:
    """Linear decay chain s0 -> s1 -> ... -> s_m with temperature-independent
    rates (a1..a6 = 0, a0 = ln k) and all mass numbers 1 (a Bateman chain)."""
    m = len(rates)
    reactants = -np.ones((m, 3), dtype=np.int32)
    products = -np.ones((m, 3), dtype=np.int32)
    for r in range(m):
        reactants[r, 0] = r
        products[r, 0] = r + 1
    coef = np.zeros((m, 7))
    coef[:, 0] = np.log(np.asarray(rates, dtype=np.float64))
    qq = np.zeros(m) if q is None else np.asarray(q, dtype=np.float64)
    return NetworkSpec(f"chain{m + 1}", np.ones(m + 1, dtype=np.int32), reactants, products,
                       coef, qq, c_v)


def reversible_pair(k_f: float, k_r: float, two_body: bool = False) -> NetworkSpec:
    """A <-> B (both mass 1), or with two_body=True 2A <-> B (A mass 1, B mass 2),
    temperature-independent rates, no heat."""
    if two_body:
        mass = np.array([1, 2])
        reactants = np.array([[0, 0, -1], [1, -1, -1]])
        products = np.array([[1, -1, -1], [0, 0, -1]])
    else:
        mass = np.array([1, 1])
        reactants = np.array([[0, -1, -1], [1, -1, -1]])
        products = np.array([[1, -1, -1], [0, -1, -1]])
    coef = np.zeros((2, 7))
    coef[:, 0] = np.log([k_f, k_r])
    return NetworkSpec("pair2" if two_body else "pair1", mass, reactants, products, coef,
                       np.zeros(2), 100.0)
