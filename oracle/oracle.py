"""ctypes binding of the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

``build()`` compiles oracle.c with gcc (-O2, no fast-math, no FMA
contraction, OpenMP) into liboracle.so next to this file.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

STATUS = {0: "OK", 1: "MAX_STEPS", 2: "STEP_UNDERFLOW", 3: "NONFINITE", 4: "BAD_INPUT"}
COUNTERS = ["n_steps", "n_rej_err", "n_newton_fail", "n_rhs", "n_jac", "n_lu", "n_solve", "order"]


def compile_source(src: str, out: str) -> str:
    """gcc -O2, no fast-math, no FMA contraction, OpenMP: src -> out (.so)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-variable", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile liboracle.so (always when force)."""
    if force or not os.path.exists(LIB):
        compile_source(SRC, LIB)
    return LIB


class _Net(C.Structure):
    _fields_ = [("n_species", C.c_int), ("n_reactions", C.c_int),
                ("mass", C.POINTER(C.c_int32)), ("reactants", C.POINTER(C.c_int32)),
                ("products", C.POINTER(C.c_int32)), ("coef", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)), ("c_v", C.c_double),
                ("screen", C.POINTER(C.c_double)), ("rounding_probe", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("t_end", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_steps", C.c_int), ("fixed_order", C.c_int), ("fixed_h", C.c_double),
                ("D_init", C.POINTER(C.c_double)), ("newton_tol_fixed", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(C.CDLL(LIB))
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Run the binding's functions against another build of the oracle
    (tests that plant a mistake in a copy of oracle.c use this)."""
    global _lib
    saved = lib()
    _lib = _bind(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def _bind(L):
    """Set the argument and result types of an oracle build's functions."""
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.orc_rates.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, dp]
    L.orc_rhs.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, dp]
    L.orc_jac.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, dp]
    L.orc_lu_factor.argtypes = [C.c_int, dp, ip]
    L.orc_lu_factor.restype = C.c_int
    L.orc_lu_solve.argtypes = [C.c_int, dp, ip, dp]
    L.orc_rescale.argtypes = [C.c_int, C.c_int, dp, C.c_double]
    L.orc_burn_cell.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, C.POINTER(_Opts),
                                C.POINTER(C.c_int32)]
    L.orc_burn_cell.restype = C.c_int
    L.orc_burn_cell_sched.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, C.POINTER(_Opts),
                                      C.POINTER(C.c_int32), dp, dp, dp,
                                      C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int)]
    L.orc_burn_cell_sched.restype = C.c_int
    L.orc_initial_step.argtypes = [C.POINTER(_Net), C.c_double, dp, dp, C.c_double,
                                   C.c_double, C.c_double]
    L.orc_initial_step.restype = C.c_double
    L.orc_error_norm.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp]
    L.orc_error_norm.restype = C.c_double
    L.orc_choose_order.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp,
                                   C.POINTER(C.c_double)]
    L.orc_choose_order.restype = C.c_int
    L.orc_burn_batch.argtypes = [C.POINTER(_Net), C.c_int64, dp, dp, dp, dp, C.POINTER(_Opts),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int]
    L.orc_burn_batch.restype = C.c_int
    L.orc_sens_batch.argtypes = [C.POINTER(_Net), C.c_int64, dp, dp, dp, dp, dp,
                                 C.POINTER(_Opts), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32), C.c_int]
    L.orc_sens_batch.restype = C.c_int
    L.orc_burn_batch_src.argtypes = [C.POINTER(_Net), C.c_int64, dp, dp, dp, dp, dp,
                                     C.POINTER(_Opts), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.c_int]
    L.orc_burn_batch_src.restype = C.c_int
    L.orc_max_threads.restype = C.c_int
    return L


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleNet:
    """Holds the network arrays alive and the C struct pointing at them."""

    def __init__(self, spec, rounding_probe: int = 0):
        """rounding_probe: test hook, 0 for every real run (see orc_net in
        oracle.c): 1 rate constants of every third reaction one ulp up, 2 the
        right-hand side's species sums in descending reaction order, 3 the
        heat term times 1/c_v."""
        spec.validate()
        self.spec = spec
        self.mass = np.ascontiguousarray(spec.mass, dtype=np.int32)
        self.reactants = np.ascontiguousarray(spec.reactants, dtype=np.int32)
        self.products = np.ascontiguousarray(spec.products, dtype=np.int32)
        self.coef = np.ascontiguousarray(spec.coef, dtype=np.float64)
        self.q = np.ascontiguousarray(spec.q, dtype=np.float64)
        self.screen = (None if spec.screen is None
                       else np.ascontiguousarray(spec.screen, dtype=np.float64))
        i32 = C.POINTER(C.c_int32)
        self.c = _Net(spec.n_species, spec.n_reactions, self.mass.ctypes.data_as(i32),
                      self.reactants.ctypes.data_as(i32), self.products.ctypes.data_as(i32),
                      _dp(self.coef), _dp(self.q), float(spec.c_v), _dp(self.screen),
                      int(rounding_probe))
        self.N = spec.n_species
        self.R = spec.n_reactions
        self.n = self.N + 1


def _lm(net: OracleNet, log_mult) -> Optional[np.ndarray]:
    if log_mult is None:
        return None
    lm = np.ascontiguousarray(log_mult, dtype=np.float64)
    assert lm.shape == (net.R,)
    return lm


def rates(net: OracleNet, T: float, log_mult=None) -> Tuple[np.ndarray, np.ndarray]:
    lam = np.zeros(net.R)
    dl = np.zeros(net.R)
    lm = _lm(net, log_mult)
    lib().orc_rates(C.byref(net.c), float(T), _dp(lm), _dp(lam), _dp(dl))
    return lam, dl


def rhs(net: OracleNet, rho: float, y, log_mult=None) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    f = np.zeros(net.n)
    lm = _lm(net, log_mult)
    lib().orc_rhs(C.byref(net.c), float(rho), _dp(y), _dp(lm), _dp(f))
    return f


def jac(net: OracleNet, rho: float, y, log_mult=None) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    J = np.zeros((net.n, net.n))
    lm = _lm(net, log_mult)
    lib().orc_jac(C.byref(net.c), float(rho), _dp(y), _dp(lm), _dp(J))
    return J


def lu_factor(A) -> Tuple[np.ndarray, np.ndarray, int]:
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.intc)
    info = lib().orc_lu_factor(n, _dp(A), piv.ctypes.data_as(C.POINTER(C.c_int)))
    return A, piv, int(info)


def lu_solve(LU, piv, b) -> np.ndarray:
    x = np.array(b, dtype=np.float64, copy=True)
    LU = np.ascontiguousarray(LU, dtype=np.float64)
    piv = np.ascontiguousarray(piv, dtype=np.intc)
    lib().orc_lu_solve(LU.shape[0], _dp(LU), piv.ctypes.data_as(C.POINTER(C.c_int)), _dp(x))
    return x


def rescale(D, k: int, rho_h: float) -> np.ndarray:
    """D: [rows >= k+1, n] backward differences; returns a rescaled copy."""
    D = np.array(D, dtype=np.float64, order="C", copy=True)
    lib().orc_rescale(D.shape[1], int(k), _dp(D), float(rho_h))
    return D


def _opts(t_end, rtol, atol, max_steps, fixed_order=0, fixed_h=0.0, D_init=None, tol=1e-12):
    return _Opts(float(t_end), float(rtol), float(atol), int(max_steps), int(fixed_order),
                 float(fixed_h), _dp(D_init), float(tol))


def burn_cell(net: OracleNet, rho: float, y0, t_end: float, rtol: float = 1e-6,
              atol: float = 1e-10, log_mult=None, max_steps: int = 100000):
    """One cell; returns (y_end, status, counters[8])."""
    y = np.array(y0, dtype=np.float64, copy=True)
    cnt = np.zeros(8, dtype=np.int32)
    lm = _lm(net, log_mult)
    o = _opts(t_end, rtol, atol, max_steps)
    st = lib().orc_burn_cell(C.byref(net.c), float(rho), _dp(y), _dp(lm), C.byref(o),
                             cnt.ctypes.data_as(C.POINTER(C.c_int32)))
    return y, int(st), cnt


def burn_cell_schedule(net: OracleNet, rho: float, y0, t_end: float, rtol: float = 1e-6,
                       atol: float = 1e-10, log_mult=None, max_steps: int = 100000):
    """One cell with its control decisions; returns (y_end, status,
    counters[8], h_init, h[n], ratio[n], order[n]) over the n accepted
    steps."""
    y = np.array(y0, dtype=np.float64, copy=True)
    cnt = np.zeros(8, dtype=np.int32)
    lm = _lm(net, log_mult)
    o = _opts(t_end, rtol, atol, max_steps)
    cap = int(max_steps)
    h = np.zeros(cap)
    ratio = np.zeros(cap)
    order = np.zeros(cap, dtype=np.int32)
    h_init = C.c_double()
    n_rec = C.c_int()
    st = lib().orc_burn_cell_sched(C.byref(net.c), float(rho), _dp(y), _dp(lm), C.byref(o),
                                   cnt.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h_init),
                                   _dp(h), _dp(ratio), order.ctypes.data_as(C.POINTER(C.c_int32)),
                                   cap, C.byref(n_rec))
    k = n_rec.value
    return y, int(st), cnt, h_init.value, h[:k], ratio[:k], order[:k]


def initial_step(net: OracleNet, rho: float, y0, t_end: float, rtol: float = 1e-6,
                 atol: float = 1e-10, log_mult=None) -> float:
    """The integrator's initial step size for y0 (-1 if f(y0) is not finite)."""
    y = np.ascontiguousarray(y0, dtype=np.float64)
    lm = _lm(net, log_mult)
    return float(lib().orc_initial_step(C.byref(net.c), float(rho), _dp(y), _dp(lm),
                                        float(t_end), float(rtol), float(atol)))


def error_norm(k: int, d, y_old, y_new, rtol: float, atol: float):
    """The order-k local error estimate of a step with corrector increment d
    from y_old to y_new; returns (err, scale)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    yo = np.ascontiguousarray(y_old, dtype=np.float64)
    yn = np.ascontiguousarray(y_new, dtype=np.float64)
    s = np.zeros(d.shape[0])
    e = lib().orc_error_norm(d.shape[0], int(k), _dp(d), _dp(yo), _dp(yn), float(rtol),
                             float(atol), _dp(s))
    return float(e), s


def choose_order(k: int, err: float, dk, dk2, scale):
    """The order / step choice after an accepted order-k step from the
    updated rows D_k, D_{k+2} and the error test's scale; returns
    (new order, step ratio)."""
    dk = np.ascontiguousarray(dk, dtype=np.float64)
    dk2 = np.ascontiguousarray(dk2, dtype=np.float64)
    s = np.ascontiguousarray(scale, dtype=np.float64)
    f = C.c_double()
    kn = lib().orc_choose_order(dk.shape[0], int(k), float(err), _dp(dk), _dp(dk2), _dp(s),
                                C.byref(f))
    return int(kn), f.value


def burn_fixed(net: OracleNet, rho: float, D_init, k: int, h: float, n_steps: int,
               log_mult=None, newton_tol: float = 1e-12):
    """Test hook: k-step BDF at constant h from the given backward
    differences (k+1 rows), n_steps steps, Newton iterated to newton_tol.
    Returns (y_end, status, counters)."""
    D_init = np.ascontiguousarray(D_init, dtype=np.float64)
    assert D_init.shape == (k + 1, net.n)
    y = np.array(D_init[0], copy=True)
    cnt = np.zeros(8, dtype=np.int32)
    lm = _lm(net, log_mult)
    o = _opts(1e300, 1e-6, 1e-10, n_steps, k, h, D_init, newton_tol)
    st = lib().orc_burn_cell(C.byref(net.c), float(rho), _dp(y), _dp(lm), C.byref(o),
                             cnt.ctypes.data_as(C.POINTER(C.c_int32)))
    return y, int(st), cnt


def burn(net: OracleNet, cells, t_end: float, rtol: float = 1e-6, atol: float = 1e-10,
         log_mult=None, max_steps: int = 100000, n_threads: int = 0, source=None):
    """Batch burn on the host.  cells: synth.Cells; source: optional constant
    per-cell source [n, C] added to the right-hand side.  Returns
    (Y[N,C], T[C], status[C], counters[8,C])."""
    Y = np.array(cells.Y, dtype=np.float64, order="C", copy=True)
    T = np.array(cells.T, dtype=np.float64, copy=True)
    rho = np.ascontiguousarray(cells.rho, dtype=np.float64)
    C_ = rho.shape[0]
    st = np.zeros(C_, dtype=np.int32)
    cnt = np.zeros((8, C_), dtype=np.int32)
    lm = _lm(net, log_mult)
    o = _opts(t_end, rtol, atol, max_steps)
    if source is not None:
        src = np.ascontiguousarray(source, dtype=np.float64)
        assert src.shape == (net.n, C_)
        rc = lib().orc_burn_batch_src(C.byref(net.c), C_, _dp(Y), _dp(rho), _dp(T), _dp(lm),
                                      _dp(src), C.byref(o), st.ctypes.data_as(C.POINTER(C.c_int32)),
                                      cnt.ctypes.data_as(C.POINTER(C.c_int32)), int(n_threads))
    else:
        rc = lib().orc_burn_batch(C.byref(net.c), C_, _dp(Y), _dp(rho), _dp(T), _dp(lm),
                                  C.byref(o), st.ctypes.data_as(C.POINTER(C.c_int32)),
                                  cnt.ctypes.data_as(C.POINTER(C.c_int32)), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the network size")
    return Y, T, st, cnt


def max_threads() -> int:
    return int(lib().orc_max_threads())


def sens(net: OracleNet, cells, t_end: float, rtol: float = 1e-6, atol: float = 1e-10,
         log_mult=None, log_mult_replay=None, want_S: bool = True, max_steps: int = 100000,
         n_threads: int = 0):
    """Record each cell's schedule with log_mult, replay it with exact
    correctors and log_mult_replay (default: log_mult), with forward
    sensitivities.  Returns (Y_end[N,C], T_end[C], status[C], counters[8,C],
    S[C,n,R] = d y_end / d p or None, n_unconv[C])."""
    Y = np.array(cells.Y, dtype=np.float64, order="C", copy=True)
    T = np.array(cells.T, dtype=np.float64, copy=True)
    rho = np.ascontiguousarray(cells.rho, dtype=np.float64)
    C_ = rho.shape[0]
    st = np.zeros(C_, dtype=np.int32)
    cnt = np.zeros((8, C_), dtype=np.int32)
    unc = np.zeros(C_, dtype=np.int32)
    S = np.zeros((C_, net.n, net.R)) if want_S else None
    lm = _lm(net, log_mult)
    lmr = _lm(net, log_mult_replay)
    o = _opts(t_end, rtol, atol, max_steps)
    i32 = C.POINTER(C.c_int32)
    rc = lib().orc_sens_batch(C.byref(net.c), C_, _dp(Y), _dp(rho), _dp(T), _dp(lm), _dp(lmr),
                              C.byref(o), st.ctypes.data_as(i32), cnt.ctypes.data_as(i32),
                              _dp(S), unc.ctypes.data_as(i32), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the network size")
    return Y, T, st, cnt, S, unc


def vjp(net: OracleNet, S, gY, gE) -> np.ndarray:
    """Per-cell gradient [R, C] of sum_i gY_i Y_i + gE E (E = c_v (T - T0))
    from forward sensitivities S [C, n, R]."""
    g = np.vstack([np.asarray(gY, dtype=np.float64),
                   net.spec.c_v * np.asarray(gE, dtype=np.float64)[None, :]])  # [n, C]
    return np.einsum("cnr,nc->rc", S, g)
