"""Python API over the C ABI: a network handle and the batched burn.

Torch tensors provide device memory and the stream; every step of the burn
runs in the HIP kernels of libburn.so.
"""
from __future__ import annotations

import ctypes as C
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
        self._arrays = [np.ascontiguousarray(spec.mass, dtype=np.int32),
                        np.ascontiguousarray(spec.reactants, dtype=np.int32),
                        np.ascontiguousarray(spec.products, dtype=np.int32),
                        np.ascontiguousarray(spec.coef, dtype=np.float64),
                        np.ascontiguousarray(spec.q, dtype=np.float64)]
        m, rs, ps, cf, q = self._arrays
        i32 = C.POINTER(C.c_int32)
        f64 = C.POINTER(C.c_double)
        desc = _lib.NetworkDesc(spec.n_species, spec.n_reactions, m.ctypes.data_as(i32),
                                rs.ctypes.data_as(i32), ps.ctypes.data_as(i32),
                                cf.ctypes.data_as(f64), q.ctypes.data_as(f64), spec.c_v)
        h = C.c_void_p()
        _lib.check(_lib.lib().bn_network_create(C.byref(desc), C.byref(h)), "bn_network_create")
        self.handle = h

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
         device: Optional[torch.device] = None
         ) -> Tuple[torch.Tensor, torch.Tensor, Optional[torch.Tensor], Optional[torch.Tensor]]:
    """Burn every cell from t = 0 to dt on the current HIP device.

    Y [N, C], rho [C], T [C] (float64; moved to the device if needed).
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
    rc = _lib.lib().burn_batch_ex(net.handle, C_, _ptr(Yd), _ptr(rhod), _ptr(Td), float(dt),
                                  float(rtol), float(atol), _ptr(lm), _ptr(st), _ptr(cnt),
                                  C.byref(opts), C.c_void_p(stream))
    _lib.check(rc, "burn_batch_ex")
    return Yd, Td, st, cnt
