"""Inversion-step form on the GPU: 512x512x128 grid (20 m cells, h = 10 m),
32 density models sharing one geometry, forward and adjoint through the
autograd wrapper.  Dot-product test per model, finite-difference gradient of
phi(m) = 1/2 ||G m - d_obs||^2 along 16 seeded directions, and a sampled
direct sum for model 0."""

import sys

import numpy as np
import pytest
import torch

from synth import PRESETS, batch_density, sample_stations

pytestmark = pytest.mark.gpu
NAMES = ("gz", "gxx", "gxy", "gxz", "gyy", "gyz")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_10160_amd as gf
    return gf


@pytest.fixture(scope="module")
def models():
    g = PRESETS["inversion"]
    m = batch_density(32, g.nx, g.ny, g.nz, seed0=400)
    m_true = batch_density(1, g.nx, g.ny, g.nz, seed0=499)
    return g, m, m_true


@pytest.mark.parametrize("prec,dot_tol,fd_tol", [("f64", 1e-13, 1e-9), ("f32", 1e-6, 1e-4)])
def test_inversion_step(gf, orc, models, prec, dot_tol, fd_tol):
    g, m_np, mt_np = models
    dt = torch.float64 if prec == "f64" else torch.float32
    note("inversion %s: plans" % prec)
    p64 = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, gf.ALL6, "f64")
    d_obs64 = p64.forward(torch.from_numpy(mt_np).cuda())          # [1][6][ny][nx]
    p64.close()
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, gf.ALL6, prec)
    op = gf.GravityOperator(p)
    m = torch.from_numpy(m_np).to("cuda", dt)
    d_obs = d_obs64.to(dt)

    note("inversion %s: forward + adjoint via autograd" % prec)
    mv = m.clone().requires_grad_(True)
    r = op(mv) - d_obs
    phi = 0.5 * (r.double() ** 2).sum()
    phi.backward()
    grad = mv.grad.double()

    # dot-product test per model: <G m_b, r_b> = <m_b, G^T r_b>
    gm = p.forward(m).double()
    rr = torch.randn(gm.shape, generator=torch.Generator(device="cuda").manual_seed(41),
                     device="cuda", dtype=torch.float64).to(dt)
    gtr = p.adjoint(rr).double()
    rr = rr.double()
    for b in range(m.shape[0]):
        lhs = float((gm[b] * rr[b]).sum())
        rhs = float((m[b].double() * gtr[b]).sum())
        assert abs(lhs - rhs) <= dot_tol * float(gm[b].norm() * rr[b].norm()), (b, lhs, rhs)

    # phi is quadratic, so the central difference is exact up to rounding:
    # (phi(m + e v) - phi(m - e v)) / (2 e) = <grad phi, v> for any e
    gen = torch.Generator(device="cuda").manual_seed(77)
    scale = float(m.double().abs().mean())
    for k in range(16):
        v = torch.randn(m.shape, generator=gen, device="cuda", dtype=torch.float64)
        eps = scale / float(v.abs().mean())
        with torch.no_grad():
            fp = 0.5 * ((p.forward((m.double() + eps * v).to(dt)) - d_obs).double() ** 2).sum()
            fm = 0.5 * ((p.forward((m.double() - eps * v).to(dt)) - d_obs).double() ** 2).sum()
        fd = float(fp - fm) / (2 * eps)
        an = float((grad * v).sum())
        note("fd %s dir %d: fd %.9e autograd %.9e" % (prec, k, fd, an))
        assert abs(fd - an) <= fd_tol * abs(an), (k, fd, an)

    # sampled direct sum for model 0
    st = sample_stations(g.nx, g.ny, 3, seed=404)
    note("inversion %s: oracle at %d stations" % (prec, len(st)))
    want = orc.forward(g, m_np[0], st)
    got = gm[0].cpu().numpy()
    tol = 1e-10 if prec == "f64" else 1e-5
    for c in range(6):
        gv = got[c][st[:, 1], st[:, 0]]
        e = float(np.linalg.norm(gv - want[:, c]) / np.linalg.norm(want[:, c]))
        note("inversion %s %s sampled rel %.2e" % (prec, NAMES[c], e))
        assert e <= tol, NAMES[c]
    p.close()
