"""The allocation-free surrogate forward (sur_forward_noalloc, for callers
that cannot allocate device memory) against sur_forward, through the C ABI:
two calls in a row on the same handle, the second with a smaller batch, each
equal to the workspace forward bit for bit (the same kernels on the same
inputs; the batch runs in chunks of samples that fit the static scratch)."""
import ctypes as C

import numpy as np
import pytest

from paper_2605_07083_amd import presets

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward():
    import torch
    assert torch.cuda.is_available()
    from paper_2605_07083_amd import surrogate as S
    L = S.lib()
    L.sur_forward_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.sur_forward_noalloc.restype = C.c_int
    X = 2048
    net = S.Surrogate(20, X, seed=3)
    W, b = presets.surrogate_test_weights(17)
    net.set_weights(W, b)
    for batch, seed in ((20, 5), (3, 6)):
        print("case: sur_forward_noalloc, batch %d x %d cells" % (batch, X), flush=True)
        q = presets.surrogate_params(batch, seed)
        p = torch.tensor(np.stack([q["gamma_emit"], q["T_K"], q["V"], q["ng"]], 1), dtype=torch.float32,
                         device="cuda:0").contiguous()
        ref = net.forward(p)
        out = torch.full((batch, S.N_OUT, X), float("nan"), dtype=torch.float32, device="cuda:0")
        rc = L.sur_forward_noalloc(net.h, C.c_void_p(p.data_ptr()), batch, C.c_void_p(out.data_ptr()))
        assert rc == 0, L.sur_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    # a batch over the handle's own max_batch runs too (the scratch, not the workspace, limits it)
    q = presets.surrogate_params(40, 7)
    p = torch.tensor(np.stack([q["gamma_emit"], q["T_K"], q["V"], q["ng"]], 1), dtype=torch.float32,
                     device="cuda:0").contiguous()
    out = torch.empty((40, S.N_OUT, X), dtype=torch.float32, device="cuda:0")
    assert L.sur_forward_noalloc(net.h, C.c_void_p(p.data_ptr()), 40, C.c_void_p(out.data_ptr())) == 0
    torch.cuda.synchronize()
    assert torch.equal(out[:20], net.forward(p[:20])) and torch.equal(out[20:], net.forward(p[20:]))
    # cells beyond the scratch array are refused before anything is launched
    big = S.Surrogate(1, 17152, seed=3)
    o = torch.empty((1, S.N_OUT, 17152), dtype=torch.float32, device="cuda:0")
    assert L.sur_forward_noalloc(big.h, C.c_void_p(p.data_ptr()), 1, C.c_void_p(o.data_ptr())) == -1
    assert b"scratch" in L.sur_last_error()
