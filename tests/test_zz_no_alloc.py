"""The allocation-free forward pass of the closure network
(lb_mlp_forward_noalloc) against the workspace entry point lb_mlp_forward:
the same kernels over the same rows, so the outputs must be identical bit
for bit.  Two calls in a row, the second with fewer rows, check that the
library-owned array is reused correctly; a batch above the maximum is
rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_workspace_entry_point():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1007_4895_amd import lb
    from paper_1007_4895_amd import workloads as W

    L = lb.lib()
    dev = torch.device("cuda:0")
    g = W.rng(1234)
    npar = lb.mlp_param_count()
    params = torch.from_numpy((0.2 * g.normal(size=npar)).astype(np.float32)).to(dev)
    stream = torch.cuda.current_stream(dev)
    nmax = lb.MLP_NOALLOC_MAX_N
    ws = torch.empty(L.lb_mlp_workspace_bytes(nmax), dtype=torch.uint8, device=dev)
    for n in (nmax, 777):
        print(f"lb_mlp_forward_noalloc n={n}", flush=True)
        x = torch.from_numpy(g.normal(size=(n, lb.MLP_NIN)).astype(np.float32)).to(dev)
        y_ref = torch.empty((n, lb.MLP_NOUT), dtype=torch.float32, device=dev)
        y_na = torch.full((n, lb.MLP_NOUT), float("nan"), dtype=torch.float32, device=dev)
        st = L.lb_mlp_forward(C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(y_ref.data_ptr()),
                              n, C.c_void_p(ws.data_ptr()), C.c_void_p(stream.cuda_stream))
        assert st == lb.LB_OK, L.lb_last_error()
        st = L.lb_mlp_forward_noalloc(C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()),
                                      C.c_void_p(y_na.data_ptr()), n, C.c_void_p(stream.cuda_stream))
        assert st == lb.LB_OK, L.lb_last_error()
        torch.cuda.synchronize()
        a, b = y_ref.cpu().numpy(), y_na.cpu().numpy()
        assert np.all(np.isfinite(b))
        np.testing.assert_array_equal(b, a)
    # above the maximum: rejected on the host, nothing launched
    x = torch.zeros((1, lb.MLP_NIN), dtype=torch.float32, device=dev)
    st = L.lb_mlp_forward_noalloc(C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()),
                                  C.c_void_p(x.data_ptr()), nmax + 1, C.c_void_p(stream.cuda_stream))
    assert st == lb.LB_EINVAL and b"LB_MLP_NOALLOC_MAX_N" in L.lb_last_error()
