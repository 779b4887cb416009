"""gf_forward_noalloc, the forward for callers that cannot allocate: called
through the C ABI it gives the same data as gf_forward with a workspace of
its own, bit for bit, on two calls in a row (the second on a smaller
input, so the fixed scratch holds the first call's values), and it refuses
a batch whose workspace exceeds the fixed scratch."""

import ctypes

import numpy as np
import pytest
import torch

from synth import Geometry, tiny_density

pytestmark = pytest.mark.gpu


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_forward_equals_forward(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_10160_amd import _native
    lib = _native.load()
    dt = torch.float64 if prec == 0 else torch.float32
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # a large input, then a smaller one with an odd row count
    cases = [(Geometry(200, 160, 24, 20.0, 25.0, 15.0, 7.0), 3, 0x1FF),
             (Geometry(37, 21, 5, 30.0, 20.0, 10.0, 5.0), 2, 0x3F)]
    base = lib.gf_debug_live_bytes()
    for g, B, mask in cases:
        h = ctypes.c_void_p()
        assert lib.gf_plan_create(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ctypes.c_uint(mask), prec, 0, sh,
                                  ctypes.byref(h)) == _native.GF_OK, lib.gf_last_error()
        try:
            need = ctypes.c_size_t()
            while True:   # the largest batch up to B whose workspace fits the scratch
                assert lib.gf_workspace_bytes(h, 0, B, ctypes.byref(need)) == _native.GF_OK
                if need.value <= 128 << 20 or B == 1:
                    break
                B -= 1
            assert need.value <= 128 << 20
            info = _native.PlanInfo()
            assert lib.gf_plan_get_info(h, ctypes.byref(info)) == _native.GF_OK
            rho = torch.from_numpy(np.stack([tiny_density(g.nx, g.ny, g.nz, seed=90 + b, block=None)
                                             for b in range(B)])).to("cuda", dt)
            want = torch.empty((B, info.n_out, g.ny, g.nx), dtype=dt, device="cuda")
            ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            assert lib.gf_forward(h, vp(rho), vp(want), B, vp(ws), need.value, sh) == _native.GF_OK
            got = torch.full_like(want, float("nan"))
            live = lib.gf_debug_live_bytes()
            assert lib.gf_forward_noalloc(h, vp(rho), vp(got), B, sh) == _native.GF_OK, lib.gf_last_error()
            assert lib.gf_debug_live_bytes() == live
            torch.cuda.synchronize()
            assert torch.equal(got, want), (g, B)
            # a batch whose workspace is beyond the scratch is refused
            big = 1
            while True:
                assert lib.gf_workspace_bytes(h, 0, big, ctypes.byref(need)) == _native.GF_OK
                if need.value > 128 << 20:
                    break
                big *= 2
            assert lib.gf_forward_noalloc(h, vp(rho), vp(got), big, sh) == _native.GF_EBUSY
            assert lib.gf_forward_noalloc(h, None, vp(got), 1, sh) == _native.GF_EINVAL
        finally:
            lib.gf_plan_destroy(h)
    assert lib.gf_debug_live_bytes() == base
