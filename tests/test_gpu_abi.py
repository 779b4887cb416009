"""The C ABI on the GPU: the plan's internal workspace (workspace NULL, up
to max_batch models) gives the same results as a caller's workspace, and
too small a workspace or too large a batch is refused with GF_EBUSY before
anything is enqueued.  Uniform nine-component, observation-level and
layered plans."""

import ctypes

import numpy as np
import pytest
import torch

from synth import Geometry, tiny_density

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_10160_amd as gf
    from paper_2005_10160_amd import _native
    _native.load()
    return gf


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("kind", ["uniform", "levels", "layered"])
def test_internal_workspace_and_busy(gf, kind):
    from paper_2005_10160_amd import _native
    lib = _native.load()
    g = Geometry(40, 130, 6, 20.0, 25.0, 15.0, 7.0)
    zed = (ctypes.c_double * 7)(*[0.0, 4.0, 9.0, 15.0, 23.0, 33.0, 46.0])
    h = ctypes.c_void_p()
    st = torch.cuda.current_stream()
    sh = ctypes.c_void_p(st.cuda_stream)
    if kind == "uniform":
        mask, rc = 0x1FF, lib.gf_plan_create(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ctypes.c_uint(0x1FF), 0, 2,
                                             sh, ctypes.byref(h))
        p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, mask, "f64")
    elif kind == "levels":
        mask, rc = 0x1, lib.gf_plan_create_levels(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 7, ctypes.c_uint(0x1), 0,
                                                  2, sh, ctypes.byref(h))
        p = gf.plan_levels(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 7, mask, "f64")
    else:
        mask, rc = 0x3F, lib.gf_plan_create_layered(g.nx, g.ny, g.nz, g.dx, g.dy, zed, g.h, ctypes.c_uint(0x3F), 0,
                                                    2, sh, ctypes.byref(h))
        p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, list(zed), g.h, mask, "f64")
    assert rc == _native.GF_OK, lib.gf_last_error()
    try:
        info = _native.PlanInfo()
        assert lib.gf_plan_get_info(h, ctypes.byref(info)) == _native.GF_OK
        assert info.max_batch == 2 and info.internal_workspace_bytes > 0
        rho = torch.from_numpy(np.stack([tiny_density(g.nx, g.ny, g.nz, seed=s, block=None) for s in (71, 72, 73)]))
        rho = rho.cuda()
        want = p.forward(rho)                                  # the binding's own workspace
        r = torch.randn(want.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(74)).cuda()
        want_g = p.adjoint(r)
        for B in (1, 2):
            d = torch.empty((B,) + tuple(want.shape[1:]), dtype=torch.float64, device="cuda")
            assert lib.gf_forward(h, vp(rho), vp(d), B, None, 0, sh) == _native.GF_OK
            gg = torch.empty((B,) + tuple(rho.shape[1:]), dtype=torch.float64, device="cuda")
            assert lib.gf_adjoint(h, vp(r), vp(gg), B, None, 0, sh) == _native.GF_OK
            torch.cuda.synchronize()
            assert torch.equal(d, want[:B]) and torch.equal(gg, want_g[:B]), B
        # batch beyond the internal workspace, and a caller's workspace one byte short
        d = torch.empty_like(want)
        assert lib.gf_forward(h, vp(rho), vp(d), 3, None, 0, sh) == _native.GF_EBUSY
        for op, fn, x, y in ((0, lib.gf_forward, rho, d), (1, lib.gf_adjoint, r, torch.empty_like(rho))):
            need = ctypes.c_size_t()
            assert lib.gf_workspace_bytes(h, op, 3, ctypes.byref(need)) == _native.GF_OK
            ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            assert fn(h, vp(x), vp(y), 3, vp(ws), need.value - 1, sh) == _native.GF_EBUSY
            assert fn(h, vp(x), vp(y), 3, vp(ws), need.value, sh) == _native.GF_OK
        torch.cuda.synchronize()
        assert torch.equal(d, want)
        # per-pass timing of the last calls
        assert lib.gf_plan_set_timing(h, 1) == _native.GF_OK
        assert lib.gf_forward(h, vp(rho), vp(d), 2, None, 0, sh) == _native.GF_OK
        ms = (ctypes.c_double * 3)()
        assert lib.gf_plan_last_pass_ms(h, 0, ms) == _native.GF_OK
        assert all(v >= 0 for v in ms) and sum(ms) > 0
    finally:
        lib.gf_plan_destroy(h)
        p.close()


def test_calls_on_two_streams_overlap_safely(gf):
    """The header's thread-safety claim: calls on different streams may
    overlap when each passes its own workspace.  A forward on one stream and
    an adjoint on another, enqueued back to back several times, give the
    results of the same calls made one after the other."""
    g = Geometry(64, 200, 12, 20.0, 25.0, 15.0, 7.0)
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 0x1FF, "f64")
    rho = torch.from_numpy(tiny_density(g.nx, g.ny, g.nz, seed=81, block=None)).cuda().unsqueeze(0)
    r = torch.randn((1,) + p.data_shape, dtype=torch.float64, generator=torch.Generator().manual_seed(82)).cuda()
    want_d = p.forward(rho)
    want_g = p.adjoint(r)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    wa = torch.empty(p.workspace_bytes("forward", 1), dtype=torch.uint8, device="cuda")
    wb = torch.empty(p.workspace_bytes("adjoint", 1), dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(4):
        d = torch.empty_like(want_d)
        gg = torch.empty_like(want_g)
        p.forward(rho, d, wa, stream=sa)
        p.adjoint(r, gg, wb, stream=sb)
        outs.append((d, gg))
    torch.cuda.synchronize()
    for d, gg in outs:
        assert torch.equal(d, want_d) and torch.equal(gg, want_g)
    p.close()


@pytest.mark.parametrize("ny,prec,mask,groups", [
    (1024, "f64", 0x3F, 1),     # column length 2048: six spectra in one launch
    (1024, "f64", 0x1FF, 2),    # eight spectra: six + two
    (2048, "f32", 0x3F, 1),     # length 4096 in FP32: six fit
    (2048, "f64", 0x3F, 2),     # length 4096 in FP64: one buffer of three, 3 + 3
    (2048, "f64", 0x1FF, 3),    # 3 + 3 + 2
    (2048, "f64", 0x181, 1),    # gz, gx, gy
])
def test_column_pass_groups(gf, ny, prec, mask, groups):
    """The plan reports how many column-pass launches a forward apply takes:
    spectra in groups of six, or of three where LDS holds one buffer of three
    spectrum rows but not two (FP64 at column length 4096)."""
    p = gf.plan(4, ny, 1, 20.0, 20.0, 20.0, 10.0, mask, prec)
    assert p.col_groups == groups
    p.close()


@pytest.mark.parametrize("kind,prec,max_batch", [("uniform", 0, 2), ("uniform", 1, 0), ("layered", 1, 1),
                                                 ("levels", 0, 1)])
def test_allocation_failure_returns_enomem_and_leaks_nothing(gf, kind, prec, max_batch):
    """Every device allocation a plan makes (layer edges, twiddles, spectra,
    plan-time scratch, the internal workspace) is made to fail in turn: plan
    creation returns GF_ENOMEM with no plan, and the device memory the
    library holds is back where it was.  The first allocation count that no
    longer fails builds a plan whose forward matches one built normally."""
    from paper_2005_10160_amd import _native
    lib = _native.load()
    g = Geometry(24, 40, 5, 20.0, 25.0, 15.0, 7.0)
    zed = (ctypes.c_double * 6)(*[0.0, 4.0, 9.0, 15.0, 23.0, 33.0])
    sh = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def create():
        h = ctypes.c_void_p(12345)
        if kind == "uniform":
            rc = lib.gf_plan_create(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ctypes.c_uint(0x1FF), prec, max_batch,
                                    sh, ctypes.byref(h))
        elif kind == "layered":
            rc = lib.gf_plan_create_layered(g.nx, g.ny, g.nz, g.dx, g.dy, zed, g.h, ctypes.c_uint(0x3F), prec,
                                            max_batch, sh, ctypes.byref(h))
        else:
            rc = lib.gf_plan_create_levels(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 3, ctypes.c_uint(0x3F), prec,
                                           max_batch, sh, ctypes.byref(h))
        return rc, h

    base = lib.gf_debug_live_bytes()
    failed = 0
    try:
        for nth in range(1, 20):
            assert lib.gf_debug_fail_alloc(nth) == _native.GF_OK
            rc, h = create()
            if rc == _native.GF_OK:
                break
            assert rc == _native.GF_ENOMEM, (nth, _native.status_name(rc), lib.gf_last_error())
            assert not h.value, nth
            assert lib.gf_debug_live_bytes() == base, nth
            failed += 1
        else:
            pytest.fail("plan creation never succeeded")
    finally:
        lib.gf_debug_fail_alloc(0)
    assert failed >= 4 + (max_batch > 0) + (prec == 1)
    try:
        assert lib.gf_debug_live_bytes() > base
        dt = torch.float64 if prec == 0 else torch.float32
        rho = torch.from_numpy(tiny_density(g.nx, g.ny, g.nz, seed=75, block=None)).to("cuda", dt).unsqueeze(0)
        info = _native.PlanInfo()
        assert lib.gf_plan_get_info(h, ctypes.byref(info)) == _native.GF_OK
        nt = info.n_levels
        d = torch.empty((1, nt, info.n_out, g.ny, g.nx), dtype=dt, device="cuda")
        need = ctypes.c_size_t()
        assert lib.gf_workspace_bytes(h, 0, 1, ctypes.byref(need)) == _native.GF_OK
        ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        assert lib.gf_forward(h, vp(rho), vp(d), 1, vp(ws), need.value, sh) == _native.GF_OK
        ps = "f64" if prec == 0 else "f32"
        if kind == "uniform":
            p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 0x1FF, ps)
        elif kind == "layered":
            p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, list(zed), g.h, 0x3F, ps)
        else:
            p = gf.plan_levels(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 3, 0x3F, ps)
        want = p.forward(rho)
        torch.cuda.synchronize()
        assert torch.equal(d.reshape(want.shape), want)
        p.close()
    finally:
        lib.gf_plan_destroy(h)
    assert lib.gf_debug_live_bytes() == base


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nan_density_propagates(gf, prec):
    """A NaN in one cell of the density is not an error: the call returns
    normally and, since every cell reaches every station, every output is
    NaN; the adjoint does the same with a NaN in the residual.  A model
    without the NaN in the same batch is unaffected."""
    dt = torch.float64 if prec == "f64" else torch.float32
    g = Geometry(48, 40, 6, 20.0, 25.0, 15.0, 7.0)
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 0x1FF, prec)
    rho = torch.from_numpy(np.stack([tiny_density(g.nx, g.ny, g.nz, seed=s, block=None) for s in (76, 77)]))
    rho = rho.to("cuda", dt)
    clean = p.forward(rho[1:])
    rho[0, 3, 17, 29] = float("nan")
    d = p.forward(rho)
    torch.cuda.synchronize()
    assert torch.isnan(d[0]).all()
    assert torch.equal(d[1:], clean)
    r = torch.randn(d.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(78)).to("cuda", dt)
    clean_g = p.adjoint(r[1:])
    r[0, 4, 10, 11] = float("nan")
    gg = p.adjoint(r)
    torch.cuda.synchronize()
    assert torch.isnan(gg[0]).all()
    assert torch.equal(gg[1:], clean_g)
    p.close()


@pytest.mark.parametrize("nx,ny,nz,prec,mask", [(40, 40, 20, "f64", 0x3F), (96, 50, 7, "f32", 0x1FF),
                                                (1024, 1024, 100, "f64", 0x3F)])
def test_resident_storage_against_eq22(gf, nx, ny, nz, prec, mask):
    """The plan's resident spectra beside the paper's counts: one real per
    frequency of the quarter plane per layer and resident component (rows
    padded to the column pass's pitch), which
    is at most about a quarter of the BTTB count of eq. 22 and far below
    the dense count of eq. 5."""
    p = gf.plan(nx, ny, nz, 20.0, 20.0, 20.0, 10.0, mask, prec)
    s = p.storage()
    i = p.info
    elem = 8 if prec == "f64" else 4
    quarter = i.n_spec * nz * (i.px // 2 + 1) * (i.py // 2 + 1) * elem
    # rows are padded to the column pass's pitch
    assert quarter <= s["resident_bytes"] <= 1.25 * quarter
    assert s["quarter_plane_per_layer"] == (i.px // 2 + 1) * (i.py // 2 + 1)
    assert s["bttb"] == (2 * nx - 1) * (2 * ny - 1) * nz
    assert s["dense"] == (nx * ny) ** 2 * nz
    assert s["resident_bytes"] < 0.3 * s["bttb_bytes"] or min(nx, ny) < 64
    assert s["resident_bytes"] < s["dense_bytes"]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_alignment(gf, prec):
    """Inputs and outputs one element into their buffers (aligned to the
    element, not to a pair of elements) take the row passes' element-wise
    loads and stores and give the same results bitwise as aligned ones; a
    caller's workspace off a 256-byte boundary, or a data pointer off its
    element, is refused with GF_EINVAL and nothing is written."""
    from paper_2005_10160_amd import _native
    lib = _native.load()
    dt = torch.float64 if prec == "f64" else torch.float32
    g = Geometry(40, 34, 5, 20.0, 25.0, 15.0, 7.0)
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, 0x3F, prec)
    rho = torch.from_numpy(tiny_density(g.nx, g.ny, g.nz, seed=81, block=None)).to("cuda", dt).unsqueeze(0)
    want = p.forward(rho)
    r = torch.randn(want.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(82)).to("cuda", dt)
    want_g = p.adjoint(r)

    def shifted(shape):
        n = int(np.prod(shape))
        return torch.empty(n + 1, dtype=dt, device="cuda")[1:].view(shape)

    rho_u, d_u = shifted(rho.shape), shifted(want.shape)
    rho_u.copy_(rho)
    r_u, g_u = shifted(r.shape), shifted(want_g.shape)
    r_u.copy_(r)
    p.forward(rho_u, out=d_u)
    p.adjoint(r_u, out=g_u)
    torch.cuda.synchronize()
    assert torch.equal(d_u, want) and torch.equal(g_u, want_g)

    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = p.workspace_bytes("forward", 1)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    d = torch.zeros_like(want)
    for off in (8, 128):
        rc = lib.gf_forward(p._h, vp(rho), vp(d), 1, ctypes.c_void_p(ws.data_ptr() + off), need, st)
        assert rc == _native.GF_EINVAL, lib.gf_last_error()
    rc = lib.gf_forward(p._h, ctypes.c_void_p(rho.data_ptr() + 2), vp(d), 1, vp(ws), need, st)
    assert rc == _native.GF_EINVAL, lib.gf_last_error()
    rc = lib.gf_adjoint(p._h, vp(r), ctypes.c_void_p(g_u.data_ptr() + 1), 1, vp(ws), ws.numel(), st)
    assert rc == _native.GF_EINVAL, lib.gf_last_error()
    torch.cuda.synchronize()
    assert not d.any()
    rc = lib.gf_forward(p._h, vp(rho), vp(d), 1, ctypes.c_void_p(ws.data_ptr() + 256), need, st)
    assert rc == _native.GF_OK, lib.gf_last_error()
    torch.cuda.synchronize()
    assert torch.equal(d, want)
    p.close()
