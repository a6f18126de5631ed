"""FP64 CPU oracle of the binary Shan-Chen capillary-filling model (test infrastructure).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package; the product (``paper_0807_0602_amd``) never does
and shares no code with it.

``liboracle.so`` is the plain C implementation in ``scf_oracle.c`` (Sec. 2-3 of the paper);
``front.py`` integrates the front equation (eq. GWE) and holds the closed forms of eqs. wash
and analy; ``physics.py`` has the equation of state and the read-outs used by the pins.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "scf_oracle.c"), os.path.join(_HERE, "scf3d_oracle.c")]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no FMA contraction, OpenMP over rows)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", tmp] + _SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Obs(C.Structure):
    _fields_ = [("t", C.c_int64), ("mass", C.c_double * 2), ("z", C.c_double),
                ("precursor", C.c_double), ("precursor_lo", C.c_double),
                ("precursor_hi", C.c_double), ("flags", C.c_int32)]

    def as_dict(self) -> dict:
        return {"t": int(self.t), "mass": (self.mass[0], self.mass[1]), "z": self.z,
                "precursor": self.precursor, "precursor_lo": self.precursor_lo,
                "precursor_hi": self.precursor_hi, "flags": int(self.flags)}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                 dp, dp, dp, dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_mask.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_threads.restype = C.c_int
        L.orc_init.argtypes = [C.c_void_p, dp, dp]
        L.orc_collide.argtypes = [C.c_void_p]
        L.orc_stream.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_time.restype = C.c_int64
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_macro.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_get_f.argtypes = [C.c_void_p, dp]
        L.orc_set_f.argtypes = [C.c_void_p, dp]
        L.orc_density.argtypes = [C.c_void_p, dp, dp]
        L.orc_observe.argtypes = [C.c_void_p, C.POINTER(Obs)]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc3_create.restype = C.c_void_p
        L.orc3_create.argtypes = [C.c_int] * 7 + [C.c_double, dp, dp, dp]
        L.orc3_destroy.argtypes = [C.c_void_p]
        L.orc3_init.argtypes = [C.c_void_p, dp, dp]
        L.orc3_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc3_time.restype = C.c_int64
        L.orc3_time.argtypes = [C.c_void_p]
        L.orc3_density.argtypes = [C.c_void_p, dp, dp]
        L.orc3_get_f.argtypes = [C.c_void_p, dp]
        L.orc3_set_f.argtypes = [C.c_void_p, dp]
        L.orc3_observe.argtypes = [C.c_void_p, dp, dp]
        L.orc3_feq.argtypes = [C.c_double] * 4 + [dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _d2(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(2))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def feq(n: float, ux: float, uy: float, alpha: float = 4.0 / 9.0) -> np.ndarray:
    """Equilibrium of eqs. feq1-feq3 for one node (9 values)."""
    out = np.zeros(9)
    lib().orc_feq(float(n), float(ux), float(uy), float(alpha), _dp(out))
    return out


class Oracle:
    """One box of the FP64 model.  Arrays are (ny, nx), x fastest."""

    def __init__(self, nx: int, ny: int, x0: int = 0, x1: int = 0, G: float = 0.9,
                 gw=(0.0, 0.0), tau=(1.0, 1.0), alpha=(4.0 / 9.0, 4.0 / 9.0), mass=(1.0, 1.0),
                 periodic_x: bool = True, solid: Optional[np.ndarray] = None):
        self.nx, self.ny, self.x0, self.x1 = int(nx), int(ny), int(x0), int(x1)
        self._keep = [_d2(gw), _d2(tau), _d2(alpha), _d2(mass)]
        self._h = lib().orc_create(self.nx, self.ny, self.x0, self.x1, int(bool(periodic_x)),
                                   float(G), *[_dp(a) for a in self._keep])
        if not self._h:
            raise ValueError("oracle: bad geometry")
        if solid is not None:
            m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
            assert m.shape == (self.ny, self.nx)
            lib().orc_set_mask(self._h, m.ctypes.data)

    @classmethod
    def from_case(cls, case, periodic_x: bool = True, x_offset: int = 0, width: Optional[int] = None):
        """Oracle for a Case; with x_offset/width, a window of columns (x clamped at its edges)."""
        g, p = case.geom, case.params
        nx = g.nx if width is None else width
        solid = getattr(g, "solid", None)
        if solid is not None:
            solid = np.asarray(solid)[:, x_offset:x_offset + nx]
        return cls(nx, g.ny, g.x0 - x_offset, g.x1 - x_offset, p.G, p.gw, p.tau, p.alpha, p.mass,
                   periodic_x=periodic_x, solid=solid)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def init(self, rhoA: np.ndarray, rhoB: np.ndarray) -> "Oracle":
        a = np.ascontiguousarray(rhoA, dtype=np.float64)
        b = np.ascontiguousarray(rhoB, dtype=np.float64)
        assert a.shape == (self.ny, self.nx) and b.shape == (self.ny, self.nx)
        lib().orc_init(self._h, _dp(a), _dp(b))
        return self

    def step(self, n: int = 1) -> "Oracle":
        lib().orc_step(self._h, int(n))
        return self

    def collide(self) -> None:
        lib().orc_collide(self._h)

    def stream(self) -> None:
        lib().orc_stream(self._h)

    @property
    def t(self) -> int:
        return int(lib().orc_time(self._h))

    def density(self) -> Tuple[np.ndarray, np.ndarray]:
        a = np.zeros((self.ny, self.nx))
        b = np.zeros((self.ny, self.nx))
        lib().orc_density(self._h, _dp(a), _dp(b))
        return a, b

    def populations(self) -> np.ndarray:
        f = np.zeros((2, 9, self.ny, self.nx))
        lib().orc_get_f(self._h, _dp(f))
        return f

    def set_populations(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (2, 9, self.ny, self.nx)
        lib().orc_set_f(self._h, _dp(f))

    def macro(self) -> dict:
        sh = (self.ny, self.nx)
        n = np.zeros((2,) + sh); j = np.zeros((2, 2) + sh); F = np.zeros((2, 2) + sh)
        U = np.zeros((2,) + sh); ueq = np.zeros((2, 2) + sh)
        lib().orc_macro(self._h, _dp(n), _dp(j), _dp(F), _dp(U), _dp(ueq))
        return {"n": n, "j": j, "F": F, "U": U, "ueq": ueq}

    def observe(self) -> dict:
        o = Obs()
        lib().orc_observe(self._h, C.byref(o))
        return o.as_dict()


# D3Q19 velocities in the oracle's order (scf3d_oracle.c)
CX3 = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])
CY3 = np.array([0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1])
CZ3 = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1])


def feq3(n: float, ux: float, uy: float, uz: float) -> np.ndarray:
    out = np.zeros(19)
    lib().orc3_feq(float(n), float(ux), float(uy), float(uz), _dp(out))
    return out


class Oracle3:
    """One 3-D box (D3Q19).  Arrays are (nz, ny, nx), x fastest."""

    def __init__(self, nx, ny, nz, x0=0, x1=0, walls_y=True, walls_z=False, G=0.9, gw=(0.0, 0.0),
                 tau=(1.0, 1.0), mass=(1.0, 1.0)):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self._keep = [_d2(gw), _d2(tau), _d2(mass)]
        self._h = lib().orc3_create(self.nx, self.ny, self.nz, int(x0), int(x1), int(bool(walls_y)),
                                    int(bool(walls_z)), float(G), *[_dp(a) for a in self._keep])
        if not self._h:
            raise ValueError("oracle3: bad geometry")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc3_destroy(h)
            self._h = None

    def init(self, rhoA, rhoB) -> "Oracle3":
        a = np.ascontiguousarray(rhoA, dtype=np.float64)
        b = np.ascontiguousarray(rhoB, dtype=np.float64)
        assert a.shape == (self.nz, self.ny, self.nx) and b.shape == a.shape
        lib().orc3_init(self._h, _dp(a), _dp(b))
        return self

    def step(self, n: int = 1) -> "Oracle3":
        lib().orc3_step(self._h, int(n))
        return self

    @property
    def t(self) -> int:
        return int(lib().orc3_time(self._h))

    def density(self):
        a = np.zeros((self.nz, self.ny, self.nx)); b = np.zeros_like(a)
        lib().orc3_density(self._h, _dp(a), _dp(b))
        return a, b

    def populations(self) -> np.ndarray:
        f = np.zeros((2, 19, self.nz, self.ny, self.nx))
        lib().orc3_get_f(self._h, _dp(f))
        return f

    def set_populations(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (2, 19, self.nz, self.ny, self.nx)
        lib().orc3_set_f(self._h, _dp(f))

    def observe(self) -> dict:
        m = np.zeros(2); z = np.zeros(1)
        lib().orc3_observe(self._h, _dp(m), _dp(z))
        return {"t": self.t, "mass": (m[0], m[1]), "z": float(z[0])}
