"""Python front end of libscf: device workspace and stream from PyTorch, calls through the C ABI.

PyTorch only provides device memory (a uint8 tensor the library carves up) and the HIP stream;
every step of the model runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from .inputs import Case, Geometry, Params


def _mask(g: Geometry) -> Optional[np.ndarray]:
    if g.solid is None:
        return None
    m = np.ascontiguousarray(np.asarray(g.solid) != 0, dtype=np.uint8)
    if m.shape != (g.ny, g.nx):
        raise ValueError("solid mask must have shape (ny, nx)")
    return m


def _geom(g: Geometry, mask: Optional[np.ndarray] = None) -> L.scf_geometry:
    # `mask` (from _mask) must stay alive until the init call has returned
    return L.scf_geometry(g.nx, g.ny, g.x0, g.x1, None if mask is None else mask.ctypes.data)


def _params(p: Params) -> L.scf_params:
    s = L.scf_params()
    s.G = p.G
    for k in range(2):
        s.gw[k] = p.gw[k]
        s.tau[k] = p.tau[k]
        s.alpha[k] = p.alpha[k]
        s.mass[k] = p.mass[k]
    return s


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _workspace(nbytes: int, device) -> torch.Tensor:
    # 256-byte aligned: the caching allocator returns 512-byte aligned blocks
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Channel:
    """One capillary (scf_init / scf_step / scf_observe)."""

    def __init__(self, geom: Geometry, params: Params, rhoA: np.ndarray, rhoB: np.ndarray,
                 device="cuda:0", stream: Optional[torch.cuda.Stream] = None):
        self.geom, self.params = geom, params
        self._m = _mask(geom)
        self._g, self._p = _geom(geom, self._m), _params(params)
        nbytes = L.scf_workspace_bytes(C.byref(self._g))
        if nbytes == 0:
            raise L.ScfError(L.SCF_EINVAL, f"invalid geometry {geom}")
        self.ws = _workspace(nbytes, device)
        self.stream = stream
        a = np.ascontiguousarray(rhoA, dtype=np.float64)
        b = np.ascontiguousarray(rhoB, dtype=np.float64)
        if a.shape != (geom.ny, geom.nx) or b.shape != (geom.ny, geom.nx):
            raise ValueError("density fields must have shape (ny, nx)")
        h = C.c_void_p()
        L.check(L.scf_init(C.byref(h), C.byref(self._g), C.byref(self._p), _dptr(a), _dptr(b),
                           C.c_void_p(self.ws.data_ptr()), nbytes, _stream_handle(stream)))
        self._h = h

    @classmethod
    def from_case(cls, case: Case, **kw) -> "Channel":
        return cls(case.geom, case.params, *case.fields(), **kw)

    def close(self) -> None:
        # at interpreter shutdown the binding may already be torn down
        if getattr(self, "_h", None) and getattr(L, "scf_destroy", None) is not None:
            L.scf_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def t(self) -> int:
        return int(L.scf_time(self._h))

    def step(self, n: int = 1, allow_unstable: bool = False) -> "Channel":
        # SCF_EUNSTABLE here is the last observation's flag, reported after the steps were enqueued
        L.check(L.scf_step(self._h, int(n)), allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        return self

    def observe(self, allow_unstable: bool = False) -> dict:
        o = L.scf_obs()
        L.check(L.scf_observe(self._h, C.byref(o)), allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        return o.as_dict()

    def density(self) -> Tuple[np.ndarray, np.ndarray]:
        a = np.zeros((self.geom.ny, self.geom.nx))
        b = np.zeros((self.geom.ny, self.geom.nx))
        L.check(L.scf_get_density(self._h, _dptr(a), _dptr(b)))
        return a, b

    def populations(self) -> np.ndarray:
        f = np.zeros((2, 9, self.geom.ny, self.geom.nx))
        L.check(L.scf_get_populations(self._h, _dptr(f)))
        return f

    def set_variant(self, variant: int) -> None:
        L.check(L.scf_set_variant(self._h, int(variant)))

    def set_tile(self, bx: int, cy: int, graph_steps: int = 64, order: int = 0, fuse: int = 1,
                 blocks_per_cu: int = 0) -> None:
        t = L.scf_tile(int(bx), int(cy), int(order), int(graph_steps), int(fuse), int(blocks_per_cu))
        L.check(L.scf_set_tile(self._h, C.byref(t)))

    def tile(self) -> dict:
        t = L.scf_tile()
        L.check(L.scf_get_tile(self._h, C.byref(t)))
        return t.as_dict()

    def autotune(self, trial_steps: int = 20, cache: Optional[str] = None) -> dict:
        """Time the candidate schedules and keep the fastest; with `cache` (a file path) reuse or
        record the choice for this geometry class and device (scf_autotune_cached)."""
        t = L.scf_tile()
        if cache is None:
            L.check(L.scf_autotune(self._h, int(trial_steps), C.byref(t)))
        else:
            L.check(L.scf_autotune_cached(self._h, int(trial_steps), str(cache).encode(), C.byref(t)))
        return t.as_dict()

    def save(self, path: str) -> None:
        L.check(L.scf_save(self._h, path.encode()))

    def load(self, path: str) -> None:
        L.check(L.scf_load(self._h, path.encode()))


class Batch:
    """Many independent channels advanced together (scf_batch_*)."""

    def __init__(self, cases: Sequence[Case], sample_every: int, max_samples: int, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None,
                 fields: Optional[Sequence[Tuple[np.ndarray, np.ndarray]]] = None):
        """`fields`: optional initial (rhoA, rhoB) per channel in place of each case's own."""
        self.cases = list(cases)
        n = len(self.cases)
        self._m = [_mask(c.geom) for c in self.cases]
        self._g = (L.scf_geometry * n)(*[_geom(c.geom, m) for c, m in zip(self.cases, self._m)])
        self._p = (L.scf_params * n)(*[_params(c.params) for c in self.cases])
        self.max_samples = int(max_samples)
        self.sample_every = int(sample_every)
        nbytes = L.scf_batch_workspace_bytes(n, self._g, self.max_samples)
        if nbytes == 0:
            raise L.ScfError(L.SCF_EINVAL, "invalid batch geometry")
        self.ws = _workspace(nbytes, device)
        if fields is None:
            fields = [c.fields() for c in self.cases]
        if len(fields) != n:
            raise ValueError("one (rhoA, rhoB) pair per case")
        for (a, b), c in zip(fields, self.cases):
            if np.shape(a) != (c.geom.ny, c.geom.nx) or np.shape(b) != (c.geom.ny, c.geom.nx):
                raise ValueError("density fields must have shape (ny, nx)")
        self._keep = [(np.ascontiguousarray(a), np.ascontiguousarray(b)) for a, b in fields]
        pa = (C.POINTER(C.c_double) * n)(*[_dptr(a) for a, _ in self._keep])
        pb = (C.POINTER(C.c_double) * n)(*[_dptr(b) for _, b in self._keep])
        h = C.c_void_p()
        L.check(L.scf_batch_init(C.byref(h), n, self._g, self._p, pa, pb, self.sample_every,
                                 self.max_samples, C.c_void_p(self.ws.data_ptr()), nbytes,
                                 _stream_handle(stream)))
        self._keep = None
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) and getattr(L, "scf_batch_destroy", None) is not None:
            L.scf_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int, allow_unstable: bool = False) -> "Batch":
        L.check(L.scf_batch_step(self._h, int(n)), allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        return self

    def observe(self, allow_unstable: bool = False):
        """(records, nsamples): records[c][s] are dicts for s < nsamples."""
        n = len(self.cases)
        buf = (L.scf_obs * (n * self.max_samples))()
        ns = C.c_int64()
        L.check(L.scf_batch_observe(self._h, buf, C.byref(ns)),
                allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        k = ns.value
        return [[buf[c * self.max_samples + s].as_dict() for s in range(k)] for c in range(n)], k

    def density(self, c: int) -> Tuple[np.ndarray, np.ndarray]:
        g = self.cases[c].geom
        a = np.zeros((g.ny, g.nx)); b = np.zeros((g.ny, g.nx))
        L.check(L.scf_batch_get_density(self._h, int(c), _dptr(a), _dptr(b)))
        return a, b

    def set_tile(self, bx: int, cy: int, graph_steps: int = 64, order: int = 0, fuse: int = 1,
                 blocks_per_cu: int = 0) -> None:
        t = L.scf_tile(int(bx), int(cy), int(order), int(graph_steps), int(fuse), int(blocks_per_cu))
        L.check(L.scf_batch_set_tile(self._h, C.byref(t)))

    def tile(self) -> dict:
        t = L.scf_tile()
        L.check(L.scf_batch_get_tile(self._h, C.byref(t)))
        return t.as_dict()

    def autotune(self, trial_steps: int = 10, cache: Optional[str] = None) -> dict:
        """As Channel.autotune, for the whole batch."""
        t = L.scf_tile()
        if cache is None:
            L.check(L.scf_batch_autotune(self._h, int(trial_steps), C.byref(t)))
        else:
            L.check(L.scf_batch_autotune_cached(self._h, int(trial_steps), str(cache).encode(), C.byref(t)))
        return t.as_dict()


class Channel3:
    """A three-dimensional (D3Q19) capillary: a slit (walls_y) or a square duct (walls_y and
    walls_z) over x in [x0, x1) (scf3_init / scf3_step / scf3_observe).  Fields are (nz, ny, nx)."""

    def __init__(self, nx: int, ny: int, nz: int, x0: int, x1: int, params: Params, rhoA: np.ndarray,
                 rhoB: np.ndarray, walls_y: bool = True, walls_z: bool = False, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        self.shape = (int(nz), int(ny), int(nx))
        self.params = params
        self._g = L.scf3_geometry(int(nx), int(ny), int(nz), int(x0), int(x1), int(bool(walls_y)),
                                  int(bool(walls_z)))
        self._p = _params(params)
        nbytes = L.scf3_workspace_bytes(C.byref(self._g))
        if nbytes == 0:
            raise L.ScfError(L.SCF_EINVAL, "invalid 3-D geometry")
        self.ws = _workspace(nbytes, device)
        a = np.ascontiguousarray(rhoA, dtype=np.float64)
        b = np.ascontiguousarray(rhoB, dtype=np.float64)
        if a.shape != self.shape or b.shape != self.shape:
            raise ValueError("density fields must have shape (nz, ny, nx)")
        h = C.c_void_p()
        L.check(L.scf3_init(C.byref(h), C.byref(self._g), C.byref(self._p), _dptr(a), _dptr(b),
                            C.c_void_p(self.ws.data_ptr()), nbytes, _stream_handle(stream)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) and getattr(L, "scf3_destroy", None) is not None:
            L.scf3_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def t(self) -> int:
        return int(L.scf3_time(self._h))

    def step(self, n: int = 1, allow_unstable: bool = False) -> "Channel3":
        L.check(L.scf3_step(self._h, int(n)), allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        return self

    def set_schedule(self, fused: bool = True, cy: int = 16) -> "Channel3":
        """One fused kernel per step walking cy rows of y per tile, or the two-kernel form."""
        L.check(L.scf3_set_schedule(self._h, int(fused), int(cy)))
        return self

    def schedule(self) -> dict:
        f, cy = C.c_int32(), C.c_int32()
        L.check(L.scf3_get_schedule(self._h, C.byref(f), C.byref(cy)))
        return {"fused": bool(f.value), "cy": int(cy.value)}

    def observe(self, allow_unstable: bool = False) -> dict:
        o = L.scf3_obs()
        L.check(L.scf3_observe(self._h, C.byref(o)), allow=(L.SCF_EUNSTABLE,) if allow_unstable else ())
        return o.as_dict()

    def density(self) -> Tuple[np.ndarray, np.ndarray]:
        a = np.zeros(self.shape)
        b = np.zeros(self.shape)
        L.check(L.scf3_get_density(self._h, _dptr(a), _dptr(b)))
        return a, b

    def populations(self) -> np.ndarray:
        f = np.zeros((2, 19) + self.shape)
        L.check(L.scf3_get_populations(self._h, _dptr(f)))
        return f
