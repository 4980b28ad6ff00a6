"""Python API over the C ABI: a network handle and the batched burn.

Torch tensors provide device memory and the stream; every step of the burn
runs in the HIP kernels of libburn.so.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
import warnings
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from .synth import NetworkSpec


class Network:
    """A network handle (device tables) created from a NetworkSpec."""

    def __init__(self, spec: NetworkSpec):
        spec.validate()
        self.spec = spec
        desc, self._arrays = _lib.network_desc(spec)
        h = C.c_void_p()
        _lib.check(_lib.lib().bn_network_create(C.byref(desc), C.byref(h)), "bn_network_create")
        self.handle = h

    def generate(self, lanes_per_cell: int = 0, cache_dir: Optional[str] = None) -> int:
        """Compile (or take from the cache) and load the network's generated
        kernel, and select it; returns its lanes per cell.  cache_dir
        defaults to default_codegen_cache()."""
        d = default_codegen_cache() if cache_dir is None else cache_dir
        _lib.check(_lib.lib().bn_network_generate(self.handle, lanes_per_cell,
                                                  d.encode() if d else None),
                   "bn_network_generate")
        return self.body[1]

    def set_body(self, body: str) -> None:
        """'table' or 'generated' (after generate())."""
        code = {"table": _lib.BODY_TABLE, "generated": _lib.BODY_GENERATED}[body]
        _lib.check(_lib.lib().bn_network_set_body(self.handle, code), "bn_network_set_body")

    @property
    def body(self) -> Tuple[str, int]:
        """(selected body, lanes per cell of the generated kernel or 0)."""
        b, l = C.c_int32(), C.c_int32()
        _lib.check(_lib.lib().bn_network_get_body(self.handle, C.byref(b), C.byref(l)),
                   "bn_network_get_body")
        return ("generated" if b.value == _lib.BODY_GENERATED else "table"), l.value

    def set_launch(self, lanes_per_cell: int, slots_per_lane: int, block_waves: int = 0) -> None:
        """Fix the launch shape (0 lanes = back to the default)."""
        _lib.check(_lib.lib().bn_network_set_launch(self.handle, lanes_per_cell, slots_per_lane,
                                                    block_waves), "bn_network_set_launch")

    def get_launch(self) -> Tuple[int, int, int]:
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.lib().bn_network_get_launch(self.handle, C.byref(a), C.byref(b),
                                                    C.byref(c)), "bn_network_get_launch")
        return a.value, b.value, c.value

    def set_persistent_launch(self, lanes_per_cell: int, slots_per_lane: int = 1,
                              waves_per_simd: int = 2, block_waves: int = 4,
                              ms_per_cell: float = 0.0) -> None:
        """Fix the persistent kernel's launch choice (0 lanes = derive it per call)."""
        _lib.check(_lib.lib().bn_network_set_persistent_launch(
            self.handle, lanes_per_cell, slots_per_lane, waves_per_simd, block_waves,
            float(ms_per_cell)), "bn_network_set_persistent_launch")

    def get_persistent_launch(self) -> Tuple[int, int, int, int]:
        """(lanes per cell, slots per lane, waves per SIMD, waves per workgroup)."""
        v = [C.c_int32() for _ in range(4)]
        _lib.check(_lib.lib().bn_network_get_persistent_launch(self.handle,
                                                               *[C.byref(x) for x in v]),
                   "bn_network_get_persistent_launch")
        return tuple(x.value for x in v)

    def cache_key(self, device=None) -> str:
        """Key of this network's tunings: a hash of its tables, its size, the
        GPU architecture and the library version."""
        import torch
        h = hashlib.sha256()
        for a in (self.spec.mass, self.spec.reactants, self.spec.products, self.spec.coef,
                  self.spec.q):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr(float(self.spec.c_v)).encode())
        if self.spec.screen is not None:
            h.update(np.ascontiguousarray(self.spec.screen).tobytes())
        dev = device if device is not None else torch.cuda.current_device()
        arch = torch.cuda.get_device_properties(dev).gcnArchName
        ver = _lib.lib().bn_version().decode()
        return (f"{h.hexdigest()[:32]}|n={self.spec.n}|R={self.spec.n_reactions}|{arch}|"
                f"{ver}")

    @property
    def n_species(self) -> int:
        return self.spec.n_species

    @property
    def n_reactions(self) -> int:
        return self.spec.n_reactions

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.lib().bn_network_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64(t, device) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    return t.contiguous()


def burn(net: Network, Y, rho, T, dt: float, rtol: float = 1e-6, atol: float = 1e-10,
         log_mult=None, *, max_steps: int = 0, lanes_per_cell: int = 0, block_waves: int = 0,
         inplace: bool = False, want_status: bool = True, want_counters: bool = True,
         device: Optional[torch.device] = None, source=None
         ) -> Tuple[torch.Tensor, torch.Tensor, Optional[torch.Tensor], Optional[torch.Tensor]]:
    """Burn every cell from t = 0 to dt on the current HIP device.

    Y [N, C], rho [C], T [C] (float64; moved to the device if needed).
    source [N+1, C] (optional): constant per-cell rates added to the
    right-hand side (burn_batch_sdc).
    Returns (Y_end, T_end, status[C] int32, counters[8, C] int32).  With
    inplace=True, Y and T (already float64 contiguous device tensors) are
    overwritten and returned.
    """
    device = device or torch.device("cuda", torch.cuda.current_device())
    if inplace:
        Yd, Td = Y, T
        assert Yd.is_cuda and Yd.dtype == torch.float64 and Yd.is_contiguous()
        assert Td.is_cuda and Td.dtype == torch.float64 and Td.is_contiguous()
    else:
        Yd = _dev_f64(Y, device).clone()
        Td = _dev_f64(T, device).clone()
    rhod = _dev_f64(rho, device)
    C_ = rhod.shape[0]
    if Yd.shape != (net.n_species, C_) or Td.shape != (C_,):
        raise ValueError(f"shapes: Y {tuple(Yd.shape)}, T {tuple(Td.shape)}, rho {tuple(rhod.shape)}")
    lm = None if log_mult is None else _dev_f64(log_mult, device)
    if lm is not None and lm.shape != (net.n_reactions,):
        raise ValueError("log_mult must have one entry per reaction")
    st = torch.empty(C_, dtype=torch.int32, device=device) if want_status else None
    cnt = torch.empty((8, C_), dtype=torch.int32, device=device) if want_counters else None
    opts = _lib.BurnOpts(int(max_steps), int(lanes_per_cell), int(block_waves), 0)
    stream = torch.cuda.current_stream(device).cuda_stream
    if source is not None:
        src = _dev_f64(source, device)
        if src.shape != (net.n_species + 1, C_):
            raise ValueError("source must be [n_species + 1, n_cells]")
        rc = _lib.lib().burn_batch_sdc(net.handle, C_, _ptr(Yd), _ptr(rhod), _ptr(Td), float(dt),
                                       float(rtol), float(atol), _ptr(lm), _ptr(src), _ptr(st),
                                       _ptr(cnt), C.byref(opts), C.c_void_p(stream))
        _lib.check(rc, "burn_batch_sdc")
        return Yd, Td, st, cnt
    rc = _lib.lib().burn_batch_ex(net.handle, C_, _ptr(Yd), _ptr(rhod), _ptr(Td), float(dt),
                                  float(rtol), float(atol), _ptr(lm), _ptr(st), _ptr(cnt),
                                  C.byref(opts), C.c_void_p(stream))
    _lib.check(rc, "burn_batch_ex")
    return Yd, Td, st, cnt


def _prep_batch(net: Network, Y, rho, T, log_mult, device, inplace, want_status, want_counters):
    if inplace:
        Yd, Td = Y, T
        for t in (Yd, Td):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("inplace needs contiguous float64 device tensors")
    else:
        Yd = _dev_f64(Y, device).clone()
        Td = _dev_f64(T, device).clone()
    rhod = _dev_f64(rho, device)
    C_ = rhod.shape[0]
    if Yd.shape != (net.n_species, C_) or Td.shape != (C_,):
        raise ValueError(f"shapes: Y {tuple(Yd.shape)}, T {tuple(Td.shape)}, rho {tuple(rhod.shape)}")
    lm = None if log_mult is None else _dev_f64(log_mult, device)
    if lm is not None and lm.shape != (net.n_reactions,):
        raise ValueError("log_mult must have one entry per reaction")
    st = torch.empty(C_, dtype=torch.int32, device=device) if want_status else None
    cnt = torch.empty((8, C_), dtype=torch.int32, device=device) if want_counters else None
    return Yd, rhod, Td, lm, st, cnt


class MultiBurn:
    """A persistent multi-network burn: up to 8 (network, cells) batches in
    one kernel launch with a device work queue.

    The device arrays are bound at construction (float64 contiguous device
    tensors, updated in place), so ``run()`` enqueues only kernels on the
    current stream (counter resets, with ``order_cells`` the queue-order
    probe and counting sort, and the burn): it allocates nothing and can be
    captured into a graph (``capture()``) and replayed.  ``order_cells``
    hands each network's cells out stiffest first (smallest initial step);
    results do not depend on it.
    """

    def __init__(self, batches, dt: float, rtol: float = 1e-6, atol: float = 1e-10, *,
                 max_steps: int = 0, block_waves: int = 0, want_status: bool = True,
                 want_counters: bool = True, order_cells: bool = True,
                 device: Optional[torch.device] = None):
        device = device or torch.device("cuda", torch.cuda.current_device())
        if len(batches) > _lib.MAX_ITEMS:
            raise ValueError(f"at most {_lib.MAX_ITEMS} batches per launch")
        self.dt, self.rtol, self.atol = float(dt), float(rtol), float(atol)
        self.opts = _lib.BurnOpts(int(max_steps), 0, int(block_waves), int(bool(order_cells)))
        self.outputs = []
        items = (_lib.BatchItem * max(1, len(batches)))()
        for j, b in enumerate(batches):
            net, Y, rho, T = b[:4]
            lm = b[4] if len(b) > 4 else None
            Yd, rhod, Td, lmd, st, cnt = _prep_batch(net, Y, rho, T, lm, device, True,
                                                     want_status, want_counters)
            self.outputs.append((Yd, Td, st, cnt, rhod, lmd))
            items[j] = _lib.BatchItem(net.handle.value, rhod.shape[0], Yd.data_ptr(),
                                      rhod.data_ptr(), Td.data_ptr(),
                                      lmd.data_ptr() if lmd is not None else None,
                                      st.data_ptr() if st is not None else None,
                                      cnt.data_ptr() if cnt is not None else None)
        self.nets = [b[0] for b in batches]  # keep the handles alive
        self.items, self.n_items = items, len(batches)
        if order_cells:
            nb = _lib.lib().burn_batch_multi_order_workspace_bytes(self.n_items, items)
        else:
            nb = _lib.lib().burn_batch_multi_workspace_bytes(max(1, self.n_items))
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        self.graph = None

    def run(self) -> None:
        stream = torch.cuda.current_stream().cuda_stream
        rc = _lib.lib().burn_batch_multi(self.n_items, self.items, self.dt, self.rtol, self.atol,
                                         C.byref(self.opts), C.c_void_p(self.workspace.data_ptr()),
                                         self.workspace.numel(), C.c_void_p(stream))
        _lib.check(rc, "burn_batch_multi")

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Capture run() into a HIP graph (replayed with ``replay()``)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()


def burn_multi(batches, dt: float, rtol: float = 1e-6, atol: float = 1e-10, **kw):
    """Burn several (net, Y, rho, T[, log_mult]) batches in one persistent
    launch; returns [(Y_end, T_end, status, counters), ...] (new tensors)."""
    device = kw.get("device") or torch.device("cuda", torch.cuda.current_device())
    own = []
    for b in batches:
        net, Y, rho, T = b[:4]
        lm = b[4] if len(b) > 4 else None
        own.append((net, _dev_f64(Y, device).clone(), _dev_f64(rho, device),
                    _dev_f64(T, device).clone(), lm))
    mb = MultiBurn(own, dt, rtol, atol, **kw)
    mb.run()
    return [(o[0], o[1], o[2], o[3]) for o in mb.outputs]


def autotune(net: Network, Y, rho, T, dt: float, rtol: float = 1e-6, atol: float = 1e-10,
             log_mult=None, *, max_steps: int = 0, device: Optional[torch.device] = None):
    """Time every launch shape on a sample of cells and make the fastest the
    network's launch choice.  Returns [(L, S, block_waves, ms or None), ...]."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    Yd, rhod, Td = _dev_f64(Y, device), _dev_f64(rho, device), _dev_f64(T, device)
    lm = None if log_mult is None else _dev_f64(log_mult, device)
    res = (_lib.TuneResult * 64)()
    nres = C.c_int32()
    stream = torch.cuda.current_stream(device).cuda_stream
    rc = _lib.lib().bn_network_autotune(net.handle, rhod.shape[0], _ptr(Yd), _ptr(rhod), _ptr(Td),
                                        float(dt), float(rtol), float(atol), _ptr(lm),
                                        int(max_steps), res, 64, C.byref(nres),
                                        C.c_void_p(stream))
    _lib.check(rc, "bn_network_autotune")
    return [(r.lanes_per_cell, r.slots_per_lane, r.block_waves, r.ms if r.status == 0 else None)
            for r in res[:nres.value]]


def autotune_persistent(net: Network, Y, rho, T, dt: float, rtol: float = 1e-6,
                        atol: float = 1e-10, log_mult=None, *, max_steps: int = 0,
                        device: Optional[torch.device] = None):
    """Time every persistent launch choice on a sample of cells and make the
    fastest the network's persistent choice.  Returns [(L, S, waves per
    SIMD, block waves, ms or None), ...]."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    Yd, rhod, Td = _dev_f64(Y, device), _dev_f64(rho, device), _dev_f64(T, device)
    lm = None if log_mult is None else _dev_f64(log_mult, device)
    res = (_lib.PersistentTuneResult * 64)()
    nres = C.c_int32()
    stream = torch.cuda.current_stream(device).cuda_stream
    rc = _lib.lib().bn_network_autotune_persistent(
        net.handle, rhod.shape[0], _ptr(Yd), _ptr(rhod), _ptr(Td), float(dt), float(rtol),
        float(atol), _ptr(lm), int(max_steps), res, 64, C.byref(nres), C.c_void_p(stream))
    _lib.check(rc, "bn_network_autotune_persistent")
    return [(r.lanes_per_cell, r.slots_per_lane, r.waves_per_simd, r.block_waves,
             r.ms if r.status == 0 else None) for r in res[:nres.value]]


def default_codegen_cache() -> str:
    """Directory of compiled generated kernels: $BURN_CODEGEN_CACHE, else the
    package's _codegen directory."""
    return os.environ.get("BURN_CODEGEN_CACHE") or os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "_codegen")


def codegen_source(spec: NetworkSpec, lanes_per_cell: int = 0) -> str:
    """The HIP source the library generates for a network."""
    desc, keep = _lib.network_desc(spec)
    n = C.c_size_t()
    _lib.check(_lib.lib().bn_codegen_source(C.byref(desc), lanes_per_cell, None, 0, C.byref(n)),
               "bn_codegen_source")
    buf = C.create_string_buffer(n.value)
    _lib.check(_lib.lib().bn_codegen_source(C.byref(desc), lanes_per_cell, buf, n.value, None),
               "bn_codegen_source")
    del keep
    return buf.value.decode()


def codegen_prebuild(spec: NetworkSpec, lanes_per_cell: int = 0,
                     cache_dir: Optional[str] = None) -> None:
    """Compile a network's generated kernel into the cache (no GPU needed)."""
    desc, keep = _lib.network_desc(spec)
    d = default_codegen_cache() if cache_dir is None else cache_dir
    os.makedirs(d, exist_ok=True)
    _lib.check(_lib.lib().bn_codegen_prebuild(C.byref(desc), lanes_per_cell, d.encode()),
               "bn_codegen_prebuild")
    del keep


def default_tune_cache() -> str:
    """$BURN_TUNE_CACHE, else ~/.cache/paper_2312_02836_amd/tune.json."""
    return os.environ.get("BURN_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2312_02836_amd", "tune.json")


def tune_cached(net: Network, Y, rho, T, dt: float, rtol: float = 1e-6, atol: float = 1e-10,
                *, cache: Optional[str] = None, device: Optional[torch.device] = None) -> dict:
    """The network's persistent launch choice from the tuning cache (a JSON
    file keyed by Network.cache_key: network hash, n, R, GPU architecture,
    library version), or, on a miss, from autotune_persistent on the given
    sample, then stored.  Applies the choice to the network and returns the
    cache entry (with "hit": True when it came from the file)."""
    path = cache or default_tune_cache()
    key = net.cache_key(device)
    entries = {}
    if os.path.exists(path):
        with open(path) as f:
            entries = json.load(f)
    e = entries.get(key)
    if e is not None:
        L_, S_, W_, bw = e["persistent"]
        net.set_persistent_launch(L_, S_, W_, bw, e.get("ms_per_cell", 0.0))
        return dict(e, hit=True)
    results = autotune_persistent(net, Y, rho, T, dt, rtol, atol, device=device)
    choice = list(net.get_persistent_launch())
    timed = [r for r in results if r[4] is not None]
    chosen = [r[4] for r in timed if list(r[:4]) == choice]
    best_ms = chosen[0] if chosen else min(r[4] for r in timed)
    n_sample = int(rho.shape[0])
    e = {"persistent": choice, "ms_per_cell": best_ms / n_sample,
         "sample_cells": n_sample, "dt": float(dt),
         "candidates": [list(r) for r in results]}
    entries[key] = e
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1)
    os.replace(tmp, path)
    return dict(e, hit=False)


class AdjointRun:
    """A sensitivity run over a batch of cells: ``forward()`` records each
    cell's schedule and replays it (end state, released energy E), then
    ``backward(gY, gE)`` returns the per-cell gradients [R, C] of
    sum_i gY_i Y_i + gE E with respect to the log-rate multipliers.  The
    workspace (schedules, checkpoints and a pool of corrected states) is
    allocated here, from torch.  The pool starts with room for
    ``states_steps`` accepted steps (None: none); the second forward call
    first grows it to the steps the first one recorded (``fit_pool()`` does
    that at any time), so that repeated runs of one batch keep every cell's
    states; cells that do not fit are recomputed from checkpoints (the same
    gradients)."""

    def __init__(self, net: Network, Y0, rho, T0, dt: float, rtol: float = 1e-6,
                 atol: float = 1e-10, log_mult=None, *, max_steps: int = 2048,
                 states_steps: Optional[int] = None, device: Optional[torch.device] = None):
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.net, self.dt, self.rtol, self.atol = net, float(dt), float(rtol), float(atol)
        self.max_steps = int(max_steps)
        self.Y0 = _dev_f64(Y0, device)
        self.T0 = _dev_f64(T0, device)
        self.rho = _dev_f64(rho, device)
        self.C = self.rho.shape[0]
        if self.Y0.shape != (net.n_species, self.C) or self.T0.shape != (self.C,):
            raise ValueError("shapes of Y0, rho, T0 do not match")
        self.lm = None if log_mult is None else _dev_f64(log_mult, device)
        self.ws_min = _lib.lib().burn_batch_adjoint_workspace_bytes(net.handle, self.C,
                                                                    self.max_steps)
        self.ws = None
        self._pool(int(states_steps or 0), device)
        self.Y = torch.empty_like(self.Y0)
        self.T = torch.empty_like(self.T0)
        self.E = torch.empty_like(self.T0)
        self.status = torch.empty(self.C, dtype=torch.int32, device=device)
        self.counters = torch.empty((8, self.C), dtype=torch.int32, device=device)
        # the replay's Newton iterations [0] and factorizations [1] per cell
        self.replay_iters = torch.empty((2, self.C), dtype=torch.int32, device=device)
        self.device = device

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _pool(self, steps: int, device) -> None:
        """(Re)allocate the workspace with a pool for `steps` accepted steps."""
        self.pool_steps = steps
        nb = self.ws_min + _lib.lib().burn_batch_adjoint_states_bytes(self.net.handle, steps)
        self.ws = None
        self.ws = torch.empty(max(nb, 8), dtype=torch.uint8, device=device)

    def recorded_steps(self) -> int:
        """Accepted steps of the cells the last forward call finished (a
        device synchronisation)."""
        ok = self.status == 0
        return int(self.counters[0][ok].sum().item())

    def fit_pool(self) -> None:
        """Grow the pool to the steps the last forward call recorded (a
        device synchronisation; the next forward call starts a new
        forward/backward pair)."""
        need = self.recorded_steps()
        if need > self.pool_steps:
            self._pool(need, self.device)

    def forward(self):
        n_fwd = getattr(self, "_n_fwd", 0)
        if n_fwd == 1:
            self.fit_pool()
        self._n_fwd = n_fwd + 1
        rc = _lib.lib().burn_batch_adjoint_forward(
            self.net.handle, self.C, _ptr(self.Y0), _ptr(self.rho), _ptr(self.T0), self.dt,
            self.rtol, self.atol, _ptr(self.lm), self.max_steps, _ptr(self.Y), _ptr(self.T),
            _ptr(self.E), _ptr(self.status), _ptr(self.counters), _ptr(self.replay_iters),
            _ptr(self.ws), self.ws.numel(), self._stream())
        _lib.check(rc, "burn_batch_adjoint_forward")
        return self.Y, self.T, self.E, self.status

    def backward(self, gY, gE) -> torch.Tensor:
        gY = _dev_f64(gY, self.device)
        gE = _dev_f64(gE, self.device)
        grad = torch.empty((self.net.n_reactions, self.C), dtype=torch.float64, device=self.device)
        rc = _lib.lib().burn_batch_adjoint_backward(
            self.net.handle, self.C, _ptr(self.Y0), _ptr(self.rho), _ptr(self.T0), self.dt,
            self.rtol, self.atol, _ptr(self.lm), self.max_steps, _ptr(gY), _ptr(gE), _ptr(grad),
            _ptr(self.status), _ptr(self.ws), self.ws.numel(), self._stream())
        _lib.check(rc, "burn_batch_adjoint_backward")
        return grad


class BurnFn(torch.autograd.Function):
    """(Y_end[N, C], E[C]) of a burn as a differentiable function of the
    network-global log-rate multipliers p[R]; the backward pass is the
    discrete adjoint and returns dL/dp summed over the cells.

        Y, E = BurnFn.apply(p, net, Y0, rho, T0, dt, rtol, atol, max_steps)
    """

    @staticmethod
    def forward(ctx, log_mult, net, Y0, rho, T0, dt, rtol=1e-6, atol=1e-10, max_steps=2048):
        run = AdjointRun(net, Y0, rho, T0, dt, rtol, atol, log_mult.detach(),
                         max_steps=max_steps, device=log_mult.device)
        Y, T, E, status = run.forward()
        n_bad = int((status != 0).sum().item())
        if n_bad:
            codes = sorted(set(status[status != 0].tolist()))
            warnings.warn(f"{n_bad} of {run.C} cells did not reach t_end (status "
                          f"{', '.join(_lib.CELL_STATUS.get(c, str(c)) for c in codes)}); they "
                          f"keep their last state and contribute no gradient", RuntimeWarning)
        ctx.run = run
        ctx.mark_non_differentiable(status)
        return Y.clone(), E.clone(), status

    @staticmethod
    def backward(ctx, gY, gE, _gstatus):
        run = ctx.run
        if gY is None:
            gY = torch.zeros_like(run.Y)
        if gE is None:
            gE = torch.zeros_like(run.E)
        grad = run.backward(gY.contiguous(), gE.contiguous())
        return grad.sum(dim=1), None, None, None, None, None, None, None, None
