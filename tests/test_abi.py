"""The C ABI library loads and exports every function include/scf.h declares (no GPU calls)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "scf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scf3?_[a-z_]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = _declared()
    for n in ("scf_init", "scf_step", "scf_observe", "scf_batch_init", "scf_batch_step",
              "scf_batch_observe", "scf_last_error", "scf_save", "scf_load", "scf3_init", "scf3_step",
              "scf3_observe"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_0807_0602_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(_lib.EXPORTED)


def test_workspace_sizes_and_validation():
    import ctypes as C
    from paper_0807_0602_amd import _lib as L
    g = L.scf_geometry(200, 24, 50, 150)
    n = L.scf_workspace_bytes(C.byref(g))
    pitch = 256
    assert n >= 38 * 24 * pitch * 4
    assert L.scf_workspace_bytes(C.byref(L.scf_geometry(2, 24, 0, 0))) == 0      # nx too small
    assert L.scf_workspace_bytes(C.byref(L.scf_geometry(200, 24, 150, 50))) == 0  # x1 < x0
    # one population buffer (18 FP32 planes) must stay within 4 GiB: 16384 x 3640 fits, x 3641 not
    assert L.scf_workspace_bytes(C.byref(L.scf_geometry(16384, 3640, 4096, 12288))) > 2 * 18 * 4 * 3640 * 16384
    assert L.scf_workspace_bytes(C.byref(L.scf_geometry(16384, 3641, 4096, 12288))) == 0
    gs = (L.scf_geometry * 2)(L.scf_geometry(200, 24, 50, 150), L.scf_geometry(96, 22, 24, 72))
    assert L.scf_batch_workspace_bytes(2, gs, 10) > n


def test_init_rejects_bad_arguments_without_touching_the_device():
    import ctypes as C
    import numpy as np
    from paper_0807_0602_amd import _lib as L
    g = L.scf_geometry(200, 24, 50, 150)
    p = L.scf_params()
    p.G = 0.9
    for k in range(2):
        p.tau[k] = 1.0; p.alpha[k] = 4 / 9; p.mass[k] = 1.0
    a = np.zeros((24, 200))
    h = C.c_void_p()
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
    # NULL workspace
    assert L.scf_init(C.byref(h), C.byref(g), C.byref(p), dp(a), dp(a), None, 0, None) == L.SCF_EINVAL
    # tau <= 1/2 is rejected before any device work
    p.tau[1] = 0.5
    assert L.scf_init(C.byref(h), C.byref(g), C.byref(p), dp(a), dp(a), C.c_void_p(256), 1 << 30,
                      None) == L.SCF_EINVAL
    assert b"tau" in L.scf_last_error()


def test_3d_workspace_and_validation():
    import ctypes as C
    from paper_0807_0602_amd import _lib as L
    g = L.scf3_geometry(64, 12, 10, 16, 48, 1, 1)
    n = L.scf3_workspace_bytes(C.byref(g))
    plane = 10 * 12 * 64
    assert n >= 78 * plane * 4 and n % 256 == 0
    assert L.scf3_workspace_bytes(C.byref(L.scf3_geometry(64, 2, 10, 16, 48, 1, 1))) == 0   # ny < 3
    assert L.scf3_workspace_bytes(C.byref(L.scf3_geometry(64, 12, 10, 48, 16, 1, 1))) == 0  # x1 < x0
    # alpha other than 4/9 is rejected before any device call
    p = L.scf_params()
    p.G = 0.9
    for k in range(2):
        p.tau[k] = 1.0; p.alpha[k] = 4.0 / 9.0; p.mass[k] = 1.0
    p.alpha[1] = 0.6
    h = C.c_void_p()
    rc = L.scf3_init(C.byref(h), C.byref(g), C.byref(p), None, None, None, 0, None)
    assert rc == L.SCF_EINVAL and b"alpha" in L.scf_last_error()
    assert L.scf3_set_schedule(None, 1, 16) == L.SCF_EINVAL


def _prototypes():
    """name -> (return type, [parameter types]) for every function prototype of include/scf.h."""
    text = open(os.path.join(ROOT, "include", "scf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"([A-Za-z_][A-Za-z0-9_ \*]*?)\b(scf3?_[a-z_0-9]+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        ret, name, params = " ".join(m.group(1).split()), m.group(2), " ".join(m.group(3).split())
        plist = [] if params in ("", "void") else [p.strip() for p in params.split(",")]
        out[name] = (ret, plist)
    return out


def test_binding_signatures_match_the_header():
    """Argument counts and scalar types of every binding entry agree with the prototypes."""
    import ctypes as C
    from paper_0807_0602_amd import _lib
    protos = _prototypes()
    assert set(protos) == set(_lib._sig), set(protos) ^ set(_lib._sig)
    scalar = {"int": C.c_int, "int32_t": C.c_int32, "int64_t": C.c_int64, "size_t": C.c_size_t,
              "float": C.c_float}
    for name, (ret, params) in protos.items():
        res, args = _lib._sig[name]
        assert len(args) == len(params), (name, params, args)
        # return type
        r = ret.replace("const ", "").strip()
        if r == "void":
            assert res is None, name
        elif r in scalar:
            assert res is scalar[r], (name, r, res)
        else:
            assert r.endswith("*") and res is C.c_char_p, (name, r, res)
        # scalar parameters map to their exact ctypes type, pointers to pointer-sized types
        for p, a in zip(params, args):
            words = p.replace("*", " * ").split()
            if "*" in words:
                assert a in (C.c_void_p, C.c_char_p) or issubclass(a, C._Pointer), (name, p, a)
            else:
                assert a is scalar[words[0]], (name, p, a)
