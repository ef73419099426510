"""The allocation-free forward pass of the warm-start network
(tfeti_mlp_forward_noalloc, a fixed device scratch array instead of the
caller's workspace), called through the C ABI: bitwise the output of
tfeti_mlp_forward on two calls in a row, the second with fewer rows (the
array keeps the first call's contents), and a clear rejection of a row count
beyond its scratch."""

import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_1926_amd import load
    load()
    return torch.device("cuda:0")


def test_noalloc_forward_matches_workspace_forward(dev):
    from paper_1205_1926_amd import _capi as A
    from paper_1205_1926_amd.warmstart import WarmNet
    net = WarmNet(W.mlp_init(3), device=str(dev))
    lib = A.load()
    st = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rng = np.random.default_rng(12)
    for n in (7000, 1500):
        X = torch.as_tensor(rng.standard_normal((n, 31)), dtype=torch.float32, device=dev)
        Y_ref = net.forward(X).clone()
        Y = torch.full((n, 21), float("nan"), dtype=torch.float32, device=dev)
        rc = lib.tfeti_mlp_forward_noalloc(C.byref(net.s), n, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), st)
        assert rc == A.TFETI_OK, (n, rc)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_ref), n
    # beyond the scratch: rejected before any launch, with a message
    big = 20000
    Xb = torch.zeros((big, 31), dtype=torch.float32, device=dev)
    Yb = torch.zeros((big, 21), dtype=torch.float32, device=dev)
    rc = lib.tfeti_mlp_forward_noalloc(C.byref(net.s), big, C.c_void_p(Xb.data_ptr()), C.c_void_p(Yb.data_ptr()), st)
    assert rc == A.TFETI_E_INVALID
    assert b"maximum" in lib.tfeti_last_error(None)
