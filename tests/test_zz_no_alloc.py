"""The allocation-free prediction (scf_sur_predict_noalloc, device inputs and outputs, scratch in a
library-owned device array) against scf_sur_predict (host arrays, workspace scratch): the same
kernels, so the outputs and the hull test agree bit for bit, on two calls in a row with the
second call smaller than the first (the array keeps the first call's contents)."""
import ctypes as C
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_0807_0602_amd",
                       "surrogate_weights_5in.npz")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0602_amd import surrogate as S
    n = S.Network.load(WEIGHTS)
    yield n
    n.close()


def _inputs(net, n, seed):
    """n rows spread over (and slightly beyond) the training hull."""
    st = net.norm()
    rng = np.random.default_rng(seed)
    lo, hi = st["lo"].astype(np.float64), st["hi"].astype(np.float64)
    span = hi - lo
    return (lo - 0.05 * span + rng.random((n, lo.size)) * 1.1 * span).astype(np.float32)


def _noalloc(net, X):
    import torch
    from paper_0807_0602_amd import _lib as L
    n = X.shape[0]
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda:0")
    Hd = torch.full((n,), 7, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    rc = L.scf_sur_predict_noalloc(net._h, C.c_void_p(Xd.data_ptr()), n, C.c_void_p(Yd.data_ptr()),
                                   C.c_void_p(Hd.data_ptr()))
    L.check(rc)
    torch.cuda.synchronize()
    return Yd.cpu().numpy(), Hd.cpu().numpy().astype(bool)


def test_noalloc_equals_predict_twice_second_smaller(net):
    for n, seed in ((3001, 1), (77, 2)):
        _say(f"case: surrogate predict_noalloc n={n} seed={seed}")
        X = _inputs(net, n, seed)
        Y_ref, in_ref = net.predict(X)
        Y, inside = _noalloc(net, X)
        assert np.isfinite(Y).all() and np.isfinite(Y_ref).all()
        assert np.array_equal(Y, Y_ref), float(np.abs(Y - Y_ref).max())
        assert np.array_equal(inside, in_ref)
        assert 0 < inside.sum() < n          # rows on both sides of the hull


def test_noalloc_rejects_too_many_rows(net):
    from paper_0807_0602_amd import _lib as L
    import torch
    n = 8192
    Xd = torch.zeros((n, 5), dtype=torch.float32, device="cuda:0")
    Yd = torch.zeros((n, 2), dtype=torch.float32, device="cuda:0")
    rc = L.scf_sur_predict_noalloc(net._h, C.c_void_p(Xd.data_ptr()), n, C.c_void_p(Yd.data_ptr()), None)
    assert rc == L.SCF_EINVAL
    assert b"scratch" in L.scf_last_error()
    # the largest call the array takes at width 256 and 5 inputs
    X = _inputs(net, 5056, 3)
    Y, _ = _noalloc(net, X)
    Y_ref, _ = net.predict(X)
    assert np.array_equal(Y, Y_ref)
