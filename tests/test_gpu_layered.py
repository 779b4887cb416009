"""GPU parity of layered (depth-stretched) meshes: layer n spans depths
[z_n, z_{n+1}] with unequal thicknesses.  The HIP path through the C ABI
(gf_plan_create_layered) against the CPU oracle's layered direct sums.

Bar as for uniform meshes: relative L2 <= 1e-10 per component in FP64 and
<= 1e-5 in FP32.
"""

import sys

import numpy as np
import pytest
import torch

from synth import Geometry, PRESETS, tiny_density, prisms_and_grf, sample_stations

pytestmark = pytest.mark.gpu

ALL9 = 0x1FF
NAMES = ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "gx", "gy")
TOL = {"f64": 1e-10, "f32": 1e-5}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_10160_amd as gf
    from paper_2005_10160_amd import _native
    _native.load()
    return gf


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def stretched(nz, top, first, ratio):
    """Edges of a mesh whose layers thicken geometrically with depth."""
    return np.concatenate([[0.0], np.cumsum(first * ratio ** np.arange(nz))]) + top


def test_layered_kernel_table(gf, orc):
    g = Geometry(12, 20, 5, 20.0, 30.0, 1.0, 8.0)
    z = stretched(g.nz, 0.0, 4.0, 1.7)
    p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, z, g.h, 0x3F, "f64")
    for n in range(g.nz):
        got = p.debug_kernel_table(n)
        want = orc.kernel_table(g, n, mode=1, zedges=z)
        for c in range(len(NAMES)):
            s = np.abs(want[c]).max()
            assert np.abs(got[c] - want[c]).max() <= 1e-12 * s, (n, NAMES[c])
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom,z", [
    (Geometry(16, 16, 6, 25.0, 25.0, 1.0, 10.0), stretched(6, 0.0, 5.0, 1.5)),
    (Geometry(13, 7, 4, 17.0, 23.0, 1.0, 5.0), np.array([0.0, 2.0, 30.0, 31.0, 90.0])),
    (Geometry(33, 5, 3, 10.0, 10.0, 1.0, 1.0), stretched(3, 12.5, 40.0, 0.5)),
])
def test_layered_forward_and_adjoint(gf, orc, geom, z, prec):
    """Thickening, thinning, very thin and very thick layers and a buried
    top, all nine components; the adjoint against the oracle's and the dot
    product."""
    note("layered %s %s edges %s" % (geom, prec, np.round(z, 2).tolist()))
    dt = torch.float64 if prec == "f64" else torch.float32
    rho = tiny_density(geom.nx, geom.ny, geom.nz, seed=41, block=None)
    p = gf.plan_layered(geom.nx, geom.ny, geom.dx, geom.dy, z, geom.h, ALL9, prec)
    d = p.forward(torch.from_numpy(rho).to("cuda", dt)).double().cpu().numpy()
    want = orc.forward_grid(geom, rho, zedges=z)
    for c in range(len(NAMES)):
        e = rel(d[c], want[c])
        assert e <= TOL[prec], (NAMES[c], e)
    rng = np.random.default_rng(42)
    r = rng.standard_normal((len(NAMES), geom.ny, geom.nx))
    g_out = p.adjoint(torch.from_numpy(r).to("cuda", dt)).double().cpu().numpy()
    wa = orc.adjoint(geom, r, ALL9, zedges=z)
    assert rel(g_out, wa) <= TOL[prec]
    lhs = float(np.sum(d * r))
    rhs = float(np.sum(rho * g_out))
    assert abs(lhs - rhs) <= (1e-13 if prec == "f64" else 1e-6) * np.linalg.norm(d) * np.linalg.norm(r)
    p.close()


def test_uniform_edges_equal_uniform_plan(gf):
    """Edges n dz give the uniform plan's operator."""
    g = Geometry(40, 30, 12, 20.0, 20.0, 20.0, 10.0)
    rho = tiny_density(g.nx, g.ny, g.nz, seed=43, block=None)
    x = torch.from_numpy(rho).cuda()
    pu = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, "f64")
    pl = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, g.dz * np.arange(g.nz + 1), g.h, ALL9, "f64")
    a = pu.forward(x).cpu().numpy()
    b = pl.forward(x).cpu().numpy()
    for c in range(len(NAMES)):
        assert rel(b[c], a[c]) <= 1e-14, NAMES[c]
    pu.close()
    pl.close()


def test_layered_paper_scale_sampled(gf, orc):
    """1024x1024x100 with layers thickening from 5 m by 3 % per layer (a
    depth-stretched inversion mesh, 2.4 km deep), 20 m cells, h = 10 m:
    sampled stations against the layered direct sum."""
    g = PRESETS["paper_scale"]
    z = stretched(g.nz, 0.0, 5.0, 1.03)
    note("layered paper scale: density")
    rho = prisms_and_grf(g.nx, g.ny, g.nz, 20, 302, 303)
    note("layered paper scale: forward")
    p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, z, g.h, ALL9, "f64")
    d = p.forward(torch.from_numpy(rho).cuda()).cpu().numpy()
    p.close()
    st = sample_stations(g.nx, g.ny, 0, seed=1)[[8, 0, 3]]
    note("layered paper scale: oracle at %d stations" % len(st))
    want = orc.forward(g, rho, st, zedges=z)
    for c in range(len(NAMES)):
        gv = d[c][st[:, 1], st[:, 0]]
        e = rel(gv, want[:, c])
        note("layered paper scale %s sampled rel %.2e" % (NAMES[c], e))
        assert e <= TOL["f64"], NAMES[c]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_layered_paper_scale_prisms_full_field(gf, orc, prec):
    """The 20 seeded prisms of the paper-scale model on the stretched mesh
    (layers 5 m x 1.03^n), every station, all nine components, against the
    oracle's merged-prism superposition through the layered depths."""
    from synth.density import paint_prisms, random_prisms
    g = PRESETS["paper_scale"]
    z = stretched(g.nz, 0.0, 5.0, 1.03)
    prisms = random_prisms(g.nx, g.ny, g.nz, 20, 302)
    rho = paint_prisms(np.zeros((g.nz, g.ny, g.nx)), prisms)
    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    note("layered prism field: oracle at all %d stations" % len(st))
    want = orc.blocks_at_stations(g, prisms, st, zedges=z).reshape(g.ny, g.nx, len(NAMES)).transpose(2, 0, 1)
    dt = torch.float64 if prec == "f64" else torch.float32
    p = gf.plan_layered(g.nx, g.ny, g.dx, g.dy, z, g.h, ALL9, prec)
    d = p.forward(torch.from_numpy(rho).to("cuda", dt)).double().cpu().numpy()
    p.close()
    for c in range(len(NAMES)):
        e = rel(d[c], want[c])
        note("layered prism field %s %s rel %.2e" % (prec, NAMES[c], e))
        assert e <= TOL[prec], (NAMES[c], e)
