"""ctypes binding of libscf.so (include/scf.h): argument marshalling only.

Every function of the C ABI is exposed under its own name with the same arguments; the
structures mirror scf_geometry, scf_params and scf_obs.  Importing this module loads the
library and raises if it is missing: the library is the only compute path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libscf.so")

SCF_OK, SCF_EINVAL, SCF_ENOMEM, SCF_EDEVICE, SCF_EUNSTABLE, SCF_ESTATE = 0, -1, -2, -3, -4, -5
SCF_VARIANT_FUSED, SCF_VARIANT_TWO_KERNEL = 0, 1

ERROR_NAMES = {SCF_EINVAL: "SCF_EINVAL", SCF_ENOMEM: "SCF_ENOMEM", SCF_EDEVICE: "SCF_EDEVICE",
               SCF_EUNSTABLE: "SCF_EUNSTABLE", SCF_ESTATE: "SCF_ESTATE"}


class scf_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_int32), ("x1", C.c_int32),
                ("solid", C.c_void_p)]


class scf_params(C.Structure):
    _fields_ = [("G", C.c_double), ("gw", C.c_double * 2), ("tau", C.c_double * 2),
                ("alpha", C.c_double * 2), ("mass", C.c_double * 2)]


class scf_obs(C.Structure):
    _fields_ = [("t", C.c_int64), ("mass", C.c_double * 2), ("z", C.c_double),
                ("precursor", C.c_double), ("precursor_lo", C.c_double),
                ("precursor_hi", C.c_double), ("flags", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {"t": int(self.t), "mass": (self.mass[0], self.mass[1]), "z": self.z,
                "precursor": self.precursor, "precursor_lo": self.precursor_lo,
                "precursor_hi": self.precursor_hi, "flags": int(self.flags)}


class scf_tile(C.Structure):
    _fields_ = [("bx", C.c_int32), ("cy", C.c_int32), ("order", C.c_int32), ("graph_steps", C.c_int32),
                ("fuse", C.c_int32), ("blocks_per_cu", C.c_int32)]

    def as_dict(self) -> dict:
        return {"bx": self.bx, "cy": self.cy, "order": self.order, "graph_steps": self.graph_steps,
                "fuse": self.fuse, "blocks_per_cu": self.blocks_per_cu}


SCF_ORDER_STRIPS, SCF_ORDER_BANDS, SCF_ORDER_XCD, SCF_ORDER_PERSIST = 0, 1, 2, 4


class scf_sur_cfg(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32), ("max_batch", C.c_int32),
                ("max_data", C.c_int64), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("seed", C.c_uint64)]


class scf3_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("x0", C.c_int32),
                ("x1", C.c_int32), ("walls_y", C.c_int32), ("walls_z", C.c_int32)]


class scf3_obs(C.Structure):
    _fields_ = [("t", C.c_int64), ("mass", C.c_double * 2), ("z", C.c_double), ("flags", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {"t": int(self.t), "mass": (self.mass[0], self.mass[1]), "z": self.z, "flags": int(self.flags)}


class ScfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libscf.so is not built ({LIB_PATH}); run __graft_entry__.build()")

lib = C.CDLL(LIB_PATH)

_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_sig = {
    "scf_workspace_bytes": (C.c_size_t, [C.POINTER(scf_geometry)]),
    "scf_init": (C.c_int, [C.POINTER(_vp), C.POINTER(scf_geometry), C.POINTER(scf_params), _dp, _dp,
                           _vp, C.c_size_t, _vp]),
    "scf_step": (C.c_int, [_vp, C.c_int64]),
    "scf_observe": (C.c_int, [_vp, C.POINTER(scf_obs)]),
    "scf_get_density": (C.c_int, [_vp, _dp, _dp]),
    "scf_get_populations": (C.c_int, [_vp, _dp]),
    "scf_set_variant": (C.c_int, [_vp, C.c_int32]),
    "scf_set_tile": (C.c_int, [_vp, C.POINTER(scf_tile)]),
    "scf_get_tile": (C.c_int, [_vp, C.POINTER(scf_tile)]),
    "scf_autotune": (C.c_int, [_vp, C.c_int32, C.POINTER(scf_tile)]),
    "scf_autotune_cached": (C.c_int, [_vp, C.c_int32, C.c_char_p, C.POINTER(scf_tile)]),
    "scf_time": (C.c_int64, [_vp]),
    "scf_save": (C.c_int, [_vp, C.c_char_p]),
    "scf_load": (C.c_int, [_vp, C.c_char_p]),
    "scf_destroy": (None, [_vp]),
    "scf_last_error": (C.c_char_p, []),
    "scf_batch_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(scf_geometry), C.c_int32]),
    "scf_batch_init": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(scf_geometry),
                                 C.POINTER(scf_params), C.POINTER(_dp), C.POINTER(_dp), C.c_int32,
                                 C.c_int32, _vp, C.c_size_t, _vp]),
    "scf_batch_step": (C.c_int, [_vp, C.c_int64]),
    "scf_batch_observe": (C.c_int, [_vp, C.POINTER(scf_obs), C.POINTER(C.c_int64)]),
    "scf_batch_get_density": (C.c_int, [_vp, C.c_int32, _dp, _dp]),
    "scf_batch_set_tile": (C.c_int, [_vp, C.POINTER(scf_tile)]),
    "scf_batch_get_tile": (C.c_int, [_vp, C.POINTER(scf_tile)]),
    "scf_batch_autotune": (C.c_int, [_vp, C.c_int32, C.POINTER(scf_tile)]),
    "scf_batch_autotune_cached": (C.c_int, [_vp, C.c_int32, C.c_char_p, C.POINTER(scf_tile)]),
    "scf_batch_destroy": (None, [_vp]),
    "scf_sur_workspace_bytes": (C.c_size_t, [C.POINTER(scf_sur_cfg)]),
    "scf_sur_create": (C.c_int, [C.POINTER(_vp), C.POINTER(scf_sur_cfg), _vp, C.c_size_t, _vp]),
    "scf_sur_param_count": (C.c_int64, [_vp]),
    "scf_sur_get_params": (C.c_int, [_vp, _fp]),
    "scf_sur_set_params": (C.c_int, [_vp, _fp]),
    "scf_sur_reset_optimizer": (C.c_int, [_vp]),
    "scf_sur_set_lr": (C.c_int, [_vp, C.c_float]),
    "scf_sur_set_data": (C.c_int, [_vp, _fp, _fp, _fp, C.c_int64]),
    "scf_sur_get_norm": (C.c_int, [_vp, _fp, _fp, _fp, _fp]),
    "scf_sur_set_norm": (C.c_int, [_vp, _fp, _fp, _fp, _fp]),
    "scf_sur_grad": (C.c_int, [_vp, _fp, _fp, _fp, C.c_int32, _fp, _fp]),
    "scf_sur_step": (C.c_int, [_vp, _fp, _fp, _fp, C.c_int32, _fp]),
    "scf_sur_train": (C.c_int, [_vp, C.c_int64, C.c_int32, _fp]),
    "scf_sur_predict": (C.c_int, [_vp, _fp, C.c_int64, _fp, C.POINTER(C.c_uint8)]),
    "scf_sur_predict_noalloc": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "scf_sur_destroy": (None, [_vp]),
    "scf3_workspace_bytes": (C.c_size_t, [C.POINTER(scf3_geometry)]),
    "scf3_init": (C.c_int, [C.POINTER(_vp), C.POINTER(scf3_geometry), C.POINTER(scf_params), _dp, _dp,
                            _vp, C.c_size_t, _vp]),
    "scf3_step": (C.c_int, [_vp, C.c_int64]),
    "scf3_set_schedule": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "scf3_get_schedule": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "scf3_observe": (C.c_int, [_vp, C.POINTER(scf3_obs)]),
    "scf3_get_density": (C.c_int, [_vp, _dp, _dp]),
    "scf3_get_populations": (C.c_int, [_vp, _dp]),
    "scf3_time": (C.c_int64, [_vp]),
    "scf3_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_sig)


def check(code: int, allow=()) -> int:
    """Raise ScfError for a negative status not listed in `allow`."""
    if code < 0 and code not in allow:
        raise ScfError(code, lib.scf_last_error().decode(errors="replace"))
    return code
