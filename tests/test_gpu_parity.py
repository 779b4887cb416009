"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Floating-point bar: relative L2 <= 1e-10 per component for the FP64 path and
<= 1e-5 for the FP32 path, against the long-double direct sum.
"""

import sys

import numpy as np
import pytest
import torch

from synth import Geometry, PRESETS, tiny_density, paper_e1_geometry, paper_e1_density, sample_stations

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5
NAMES = ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "gx", "gy")
NC = len(NAMES)
ALL9 = 0x1FF
TENSOR = (1, 2, 3, 4, 5, 6)
VECTOR = (0, 7, 8)   # gz, gx, gy


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


def run_forward(gf, g, rho, mask=ALL9, prec="f64"):
    dt = torch.float64 if prec == "f64" else torch.float32
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, mask, prec)
    d = p.forward(torch.from_numpy(np.ascontiguousarray(rho)).to("cuda", dt))
    torch.cuda.synchronize()
    out = d.double().cpu().numpy()
    p.close()
    return out


# --------------------------------------------------------------- kgen ----
@pytest.mark.parametrize("geom,layers", [
    (PRESETS["tiny"], range(8)),
    (Geometry(12, 20, 5, 20.0, 30.0, 10.0, 8.0), range(5)),
    (Geometry(64, 48, 40, 25.0, 25.0, 20.0, 10.0), (0, 7, 39)),
])
def test_kernel_table_matches_oracle(gf, orc, geom, layers):
    """Every entry of the generated table (closed form near, Gauss-Legendre
    far) against the oracle's closed form / 8^3-rule reference."""
    note("kernel table %s" % (geom,))
    p = gf.plan(geom.nx, geom.ny, geom.nz, geom.dx, geom.dy, geom.dz, geom.h, 0x3F, "f64")
    for n in layers:
        got = p.debug_kernel_table(n)
        want = orc.kernel_table(geom, n, mode=1)
        for c in range(NC):
            s = np.abs(want[c]).max()
            diff = np.abs(got[c] - want[c])
            assert diff.max() <= 1e-12 * s, (n, NAMES[c], diff.max() / s)
            assert np.all(diff <= 1e-9 * np.abs(want[c]) + 1e-13 * s), (n, NAMES[c])
    p.close()


def test_resident_spectrum_is_dft_of_oracle_table(gf, orc):
    """The quarter-plane spectra equal numpy's DFT of the oracle's table placed
    in the circulant (unit G); the other part of each spectrum is zero.  The
    plan holds eight spectra, stored in two groups."""
    g = Geometry(12, 10, 3, 20.0, 30.0, 15.0, 9.0)
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9 & ~0x40, "f64")
    px, py = p.info.px, p.info.py
    G = orc.grav_const()
    a = np.arange(-(g.nx - 1), g.nx) % px
    b = np.arange(-(g.ny - 1), g.ny) % py
    for n in range(g.nz):
        t = orc.kernel_table(g, n, mode=1) / G
        for c, name in enumerate(NAMES):
            if name == "gzz":
                continue
            emb = np.zeros((py, px))
            emb[np.ix_(b, a)] = t[c]
            kh = np.fft.fft2(emb)            # [ky][kx]
            imag = name in ("gxz", "gyz", "gx", "gy")
            want = (kh.imag if imag else kh.real)[: py // 2 + 1, : px // 2 + 1].T
            other = (kh.real if imag else kh.imag)
            s = np.abs(kh).max()
            assert np.abs(other).max() <= 1e-12 * s, name
            got = p.debug_spectrum(name, n)
            assert np.abs(got - want).max() <= 1e-12 * s, (n, name)
    p.close()


# ------------------------------------------------------------ forward ----
def test_forward_tiny_fp64(gf, orc):
    g = PRESETS["tiny"]
    rho = tiny_density(g.nx, g.ny, g.nz)
    got = run_forward(gf, g, rho)
    want = orc.forward_grid(g, rho)
    for c in range(NC):
        e = rel(got[c], want[c])
        note("tiny fp64 %s rel %.2e" % (NAMES[c], e))
        assert e <= TOL64, NAMES[c]


@pytest.mark.parametrize("geom", [
    Geometry(12, 20, 5, 20.0, 30.0, 10.0, 8.0),
    Geometry(20, 12, 5, 30.0, 20.0, 10.0, 8.0),
    Geometry(13, 7, 3, 17.0, 23.0, 11.0, 5.0),
    Geometry(33, 5, 2, 10.0, 10.0, 40.0, 1.0),
    Geometry(1, 1, 1, 10.0, 10.0, 10.0, 5.0),
    Geometry(1, 9, 4, 10.0, 20.0, 5.0, 2.5),
    Geometry(6, 1, 3, 15.0, 10.0, 5.0, 2.5),
    Geometry(9, 8, 1, 25.0, 25.0, 2.0, 0.5),
])
def test_forward_ragged_and_anisotropic(gf, orc, geom):
    """Non-square, non-power-of-two, single-cell and single-row grids with
    unequal cell sides: catches swapped axes and embedding/crop errors."""
    note("ragged %s" % (geom,))
    rho = tiny_density(geom.nx, geom.ny, geom.nz, seed=17, block=None)
    got = run_forward(gf, geom, rho)
    want = orc.forward_grid(geom, rho)
    # With one column (nx = 1) or one row (ny = 1) every station lies on a
    # symmetry plane of every cell, where gxy and gxz (or gyz) vanish: the
    # oracle's values there are rounding noise, so tensor components are
    # measured against the size of the whole tensor (gx and gy, which vanish
    # there too, against the size of the field vector).
    tensor = max(np.linalg.norm(want[c]) for c in TENSOR)
    vector = max(np.linalg.norm(want[c]) for c in VECTOR)
    for c in range(NC):
        size = tensor if c in TENSOR else vector
        ref = np.linalg.norm(want[c]) if c == 0 else max(np.linalg.norm(want[c]), 1e-6 * size)
        assert np.linalg.norm(got[c] - want[c]) <= TOL64 * ref, NAMES[c]


# the last three need seven or eight spectra: two column-pass groups, the
# second of one or two spectra
@pytest.mark.parametrize("names", [("gz",), ("gzz",), ("gxy", "gyz"), ("gz", "gzz"), ("gxz", "gyy", "gzz"),
                                   ("gz", "gxx", "gxy", "gxz", "gyy", "gyz"), ("gx",), ("gy",),
                                   ("gz", "gx", "gy"), ("gyz", "gx", "gzz"),
                                   ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gx"),
                                   ("gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "gx", "gy"), NAMES])
def test_forward_component_subsets(gf, orc, names):
    g = Geometry(10, 14, 4, 20.0, 25.0, 15.0, 7.0)
    rho = tiny_density(g.nx, g.ny, g.nz, seed=3, block=None)
    mask = sum(1 << NAMES.index(n) for n in names)
    got = run_forward(gf, g, rho, mask)
    want = orc.forward_grid(g, rho)
    assert got.shape[0] == len(names)
    for i, n in enumerate(sorted(names, key=NAMES.index)):
        assert rel(got[i], want[NAMES.index(n)]) <= TOL64, n


def test_forward_tiny_fp32(gf, orc):
    g = PRESETS["tiny"]
    rho = tiny_density(g.nx, g.ny, g.nz)
    got = run_forward(gf, g, rho, prec="f32")
    want = orc.forward_grid(g, rho)
    for c in range(NC):
        e = rel(got[c], want[c])
        note("tiny fp32 %s rel %.2e" % (NAMES[c], e))
        assert e <= TOL32, NAMES[c]


def test_batch_equals_single(gf):
    g = Geometry(24, 16, 6, 20.0, 20.0, 20.0, 10.0)
    rho = np.stack([tiny_density(g.nx, g.ny, g.nz, seed=s, block=None) for s in (1, 2, 3)])
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, "f64")
    both = p.forward(torch.from_numpy(rho).cuda()).cpu().numpy()
    for b in range(3):
        one = p.forward(torch.from_numpy(rho[b]).cuda()).cpu().numpy()
        assert np.array_equal(both[b], one)
    p.close()


# column lengths 256, 512 and 1024: several column units per workgroup and
# one to four waves per column in the wave split; 3 models (not a multiple of
# the columns per workgroup) and 37 layers (Nyquist chunks of 2 layers, the
# last one short)
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("nx,ny", [(100, 120), (70, 200), (60, 300)])
def test_wave_split_batches(gf, orc, nx, ny, prec, tol):
    g = Geometry(nx, ny, 37, 20.0, 25.0, 15.0, 7.0)
    dt = torch.float64 if prec == "f64" else torch.float32
    rho = np.stack([tiny_density(g.nx, g.ny, g.nz, seed=s, block=None) for s in (4, 5, 6)])
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, prec)
    note("wave split %dx%dx%d %s: batch of 3" % (nx, ny, g.nz, prec))
    both = p.forward(torch.from_numpy(rho).to("cuda", dt)).double().cpu().numpy()
    for b in range(3):
        one = p.forward(torch.from_numpy(rho[b]).to("cuda", dt)).double().cpu().numpy()
        assert np.array_equal(both[b], one), b
    st = np.array([(0, 0), (nx - 1, ny - 1), (nx // 2, ny // 2), (nx // 3, (2 * ny) // 3)])
    want = orc.forward(g, rho[1], st)
    for c in range(NC):
        gv = both[1][c][st[:, 1], st[:, 0]]
        e = rel(gv, want[:, c])
        assert e <= tol, (NAMES[c], e)
    rng = np.random.default_rng(nx + ny)
    r = rng.uniform(-1.0, 1.0, size=(3, NC, ny, nx))
    gt = p.adjoint(torch.from_numpy(r).to("cuda", dt)).double().cpu().numpy()
    for b in range(3):
        one = p.adjoint(torch.from_numpy(r[b]).to("cuda", dt)).double().cpu().numpy()
        assert np.array_equal(gt[b], one), b
    lhs = float(np.sum(both * r))
    rhs = float(np.sum(rho * gt))
    dtol = 1e-13 if prec == "f64" else 1e-6
    assert abs(lhs - rhs) <= dtol * np.linalg.norm(both) * np.linalg.norm(r), (lhs, rhs)
    p.close()


# batches of models run the column passes with the groups of a workgroup on
# one column unit, its spectrum rows staged once (column lengths 256 and 512
# in both precisions, 1024 in FP32): 4 models fill the groups, 9 leave some
# idle; 21 layers (Nyquist chunks, the last one short)
@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("nx,ny", [(90, 110), (50, 200), (64, 400)])
@pytest.mark.parametrize("nb", [4, 9])
def test_shared_spectrum_batches(gf, orc, nx, ny, nb, prec, tol):
    g = Geometry(nx, ny, 21, 20.0, 25.0, 15.0, 7.0)
    dt = torch.float64 if prec == "f64" else torch.float32
    rho = np.stack([tiny_density(g.nx, g.ny, g.nz, seed=40 + s, block=None) for s in range(nb)])
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, prec)
    note("shared spectra %dx%dx%d %s: batch of %d" % (nx, ny, g.nz, prec, nb))
    both = p.forward(torch.from_numpy(rho).to("cuda", dt)).double().cpu().numpy()
    for b in (0, nb // 2, nb - 1):
        one = p.forward(torch.from_numpy(rho[b]).to("cuda", dt)).double().cpu().numpy()
        assert np.array_equal(both[b], one), b
    st = np.array([(0, 0), (nx - 1, ny - 1), (nx // 2, ny // 3), (nx // 5, (3 * ny) // 4)])
    bl = nb - 1
    want = orc.forward(g, rho[bl], st)
    for c in range(NC):
        e = rel(both[bl][c][st[:, 1], st[:, 0]], want[:, c])
        assert e <= tol, (NAMES[c], e)
    rng = np.random.default_rng(7 * nx + ny + nb)
    r = rng.uniform(-1.0, 1.0, size=(nb, NC, ny, nx))
    gt = p.adjoint(torch.from_numpy(r).to("cuda", dt)).double().cpu().numpy()
    for b in (0, nb - 1):
        one = p.adjoint(torch.from_numpy(r[b]).to("cuda", dt)).double().cpu().numpy()
        assert np.array_equal(gt[b], one), b
    lhs = float(np.sum(both * r))
    rhs = float(np.sum(rho * gt))
    dtol = 1e-13 if prec == "f64" else 1e-6
    assert abs(lhs - rhs) <= dtol * np.linalg.norm(both) * np.linalg.norm(r), (lhs, rhs)
    p.close()


def test_deterministic(gf):
    g = Geometry(40, 30, 12, 20.0, 20.0, 20.0, 10.0)
    rho = tiny_density(g.nx, g.ny, g.nz, seed=9, block=None)
    a = run_forward(gf, g, rho)
    b = run_forward(gf, g, rho)
    assert np.array_equal(a, b)


def test_paper_validation_model(gf, orc):
    """Section 3.1: the fast result against the exact merged-prism field of
    the 300 m cube; the paper reports a residual ~13 orders below the field."""
    g = paper_e1_geometry()
    rho = paper_e1_density()
    got = run_forward(gf, g, rho)
    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    want = orc.blocks_at_stations(g, [(17, 23, 17, 23, 10, 16, 300.0)], st)
    want = want.reshape(g.ny, g.nx, NC).transpose(2, 0, 1)
    worst = 0.0
    for c in range(NC):   # Fig. 6-7 include the first derivatives
        e = rel(got[c], want[c])
        worst = max(worst, e)
        note("paper model %s rel %.2e" % (NAMES[c], e))
    assert worst <= 1e-12


# ------------------------------------------------------------ adjoint ----
def test_adjoint_matches_oracle(gf, orc):
    g = Geometry(9, 7, 4, 30.0, 40.0, 25.0, 15.0)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((NC, g.ny, g.nx))
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, "f64")
    got = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy()
    want = orc.adjoint(g, r, ALL9)
    assert rel(got, want) <= TOL64
    p.close()


@pytest.mark.parametrize("names", [("gz",), ("gzz",), ("gxx", "gzz"), ("gxz", "gyz", "gxy"), ("gx",),
                                   ("gy", "gzz"), ("gz", "gx", "gy"),
                                   ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gy")])
def test_adjoint_component_subsets(gf, orc, names):
    g = Geometry(11, 6, 3, 20.0, 30.0, 10.0, 5.0)
    mask = sum(1 << NAMES.index(n) for n in names)
    order = sorted(names, key=NAMES.index)
    rng = np.random.default_rng(6)
    r_out = rng.standard_normal((len(order), g.ny, g.nx))
    r_full = np.zeros((NC, g.ny, g.nx))
    for i, n in enumerate(order):
        r_full[NAMES.index(n)] = r_out[i]
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, mask, "f64")
    got = p.adjoint(torch.from_numpy(r_out).cuda()).cpu().numpy()
    want = orc.adjoint(g, r_full, mask)
    assert rel(got, want) <= TOL64
    p.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_dot_product(gf, prec, tol):
    g = Geometry(48, 40, 10, 20.0, 25.0, 15.0, 10.0)
    dt = torch.float64 if prec == "f64" else torch.float32
    gen = torch.Generator(device="cpu").manual_seed(11)
    m = torch.randn((2, g.nz, g.ny, g.nx), generator=gen, dtype=torch.float64)
    r = torch.randn((2, NC, g.ny, g.nx), generator=gen, dtype=torch.float64)
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, prec)
    gm = p.forward(m.to("cuda", dt)).double().cpu()
    gtr = p.adjoint(r.to("cuda", dt)).double().cpu()
    lhs = float((gm * r).sum())
    rhs = float((m * gtr).sum())
    scale = float(gm.norm() * r.norm())
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs)
    p.close()


# --------------------------------------------------------- full sizes ----
_TABULATED = {}


def tabulated_oracle(orc, key, g, rho, st, mask):
    """The oracle's tabulated direct sum (eq. 3 over each layer's offset
    table), computed once per module for both precisions."""
    if key not in _TABULATED:
        import time
        t0 = time.time()
        note("%s: oracle tabulated sum at %d stations (%d threads)" % (key, len(st), orc.max_threads()))
        _TABULATED[key] = orc.forward_tabulated(g, rho, st, mask=mask)
        note("%s: oracle done in %.1f s" % (key, time.time() - t0))
    return _TABULATED[key]


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_medium_grid_every_station(gf, orc, prec, tol):
    """256x256x64, 25x25x20 m cells, h = 10 m: the complete model (6 prisms
    plus the Gaussian random field) at all 65 536 stations, all nine
    components, against the oracle's tabulated direct sum."""
    from synth import prisms_and_grf
    g = PRESETS["medium"]
    rho = prisms_and_grf(g.nx, g.ny, g.nz, 6, 202, 203)
    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    want = tabulated_oracle(orc, "medium", g, rho, st, ALL9)
    want = want.reshape(g.ny, g.nx, NC).transpose(2, 0, 1)
    note("medium grid %s: forward" % prec)
    got = run_forward(gf, g, rho, prec=prec)
    for c in range(NC):
        e = rel(got[c], want[c])
        note("medium %s %s every station rel %.2e" % (prec, NAMES[c], e))
        assert e <= tol, NAMES[c]


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_paper_scale_1024_stations(gf, orc, prec, tol):
    """1024x1024x100, 20 m cells, h = 10 m, the complete model (20 prisms plus
    the Gaussian random field) in the launch configuration the benchmark
    times (six components, batch 1): 1024 seeded stations (corners, edge
    midpoints, centre and 1015 random ones) against the oracle's tabulated
    direct sum."""
    from synth import prisms_and_grf
    g = PRESETS["paper_scale"]
    note("paper scale %s: density" % prec)
    rho = prisms_and_grf(g.nx, g.ny, g.nz, 20, 302, 303)
    st = sample_stations(g.nx, g.ny, 1015, seed=303)
    assert len(st) == 1024
    want = tabulated_oracle(orc, "paper_scale", g, rho, st, 0x3F)
    note("paper scale %s: forward" % prec)
    got = run_forward(gf, g, rho, mask=0x3F, prec=prec)
    for c in range(6):
        gv = got[c][st[:, 1], st[:, 0]]
        e = rel(gv, want[:, c])
        note("paper scale %s %s at 1024 stations rel %.2e" % (prec, NAMES[c], e))
        assert e <= tol, NAMES[c]


# every transform length the library instantiates: nx (ny) = 2^k + 1 makes
# the circulant length Px (Py) = 4 * 2^k, so these pairs reach row lengths
# Px/2 = 8 ... 2048 and column lengths Py = 16 ... 4096
SWEEP = [(9, 5), (5, 9), (33, 17), (17, 33), (129, 65), (65, 129), (513, 257), (257, 513),
         (1025, 3), (3, 1025)]


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("nx,ny", SWEEP)
def test_transform_length_sweep(gf, orc, nx, ny, prec, tol):
    """Forward and adjoint at every row and column transform length against
    the direct sum at sampled stations (corners, centre, an off-centre
    station; nz = 3, all nine components).  The FP64 column pass of length
    4096 holds three spectra per launch in LDS, with one spectrum buffer:
    there the eight spectra run as column-pass groups of three, three and
    two."""
    g = Geometry(nx, ny, 3, 20.0, 25.0, 15.0, 7.0)
    rng = np.random.default_rng(nx * 7919 + ny)
    rho = rng.uniform(-500.0, 500.0, size=(g.nz, ny, nx))
    note("sweep %dx%d %s: forward" % (nx, ny, prec))
    got = run_forward(gf, g, rho, mask=ALL9, prec=prec)
    st = np.array([(0, 0), (nx - 1, ny - 1), (nx // 2, ny // 2), (nx // 3, (2 * ny) // 3), (nx - 1, 0)])
    want = orc.forward(g, rho, st)
    for c in range(NC):
        gv = got[c][st[:, 1], st[:, 0]]
        # components that vanish on a symmetry line of a thin grid are
        # compared against the size of the whole tensor (or field vector)
        scale = np.linalg.norm(want[:, list(TENSOR if c in TENSOR else VECTOR)])
        e = float(np.linalg.norm(gv - want[:, c]) / max(np.linalg.norm(want[:, c]), 1e-3 * scale))
        assert e <= tol, (NAMES[c], e)
    # adjoint of a random residual at sampled cells
    dt = torch.float64 if prec == "f64" else torch.float32
    r = rng.uniform(-1.0, 1.0, size=(NC, ny, nx))
    p = gf.plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, ALL9, prec)
    gt = p.adjoint(torch.from_numpy(r).to("cuda", dt)).double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    cells = np.array([(0, 0, 0), (nx - 1, ny - 1, g.nz - 1), (nx // 2, ny // 3, 1)])
    wa = orc.adjoint(g, r, ALL9, cells)
    ga = gt[cells[:, 2], cells[:, 1], cells[:, 0]]
    e = rel(ga, wa)
    note("sweep %dx%d %s: adjoint rel %.2e" % (nx, ny, prec, e))
    assert e <= tol


@pytest.mark.parametrize("prec,mask", [("f32", 0x3F), ("f64", 0x1), ("f64", 0x3F)])
def test_largest_grid(gf, orc, prec, mask):
    """nx = ny = 2048, the largest grid (circulant 4096 x 4096, row and
    column transforms of the longest lengths together), three layers: FP32
    with six components, FP64 with gz alone and FP64 with six components
    (column-pass groups of three spectra with one spectrum buffer at this
    length) against the direct sum at sampled stations."""
    g = Geometry(2048, 2048, 3, 10.0, 10.0, 10.0, 5.0)
    rng = np.random.default_rng(2048)
    rho = rng.uniform(-500.0, 500.0, size=(g.nz, g.ny, g.nx))
    note("largest grid %s %s: forward" % (prec, hex(mask)))
    got = run_forward(gf, g, rho, mask=mask, prec=prec)
    st = sample_stations(g.nx, g.ny, 2, seed=2049)
    note("largest grid: oracle at %d stations" % len(st))
    want = orc.forward(g, rho, st)
    comps = [c for c in range(9) if mask >> c & 1]
    tol = TOL64 if prec == "f64" else TOL32
    for i, c in enumerate(comps):
        gv = got[i][st[:, 1], st[:, 0]]
        e = rel(gv, want[:, c])
        note("largest grid %s %s sampled rel %.2e" % (prec, NAMES[c], e))
        assert e <= tol, (NAMES[c], e)


_PRISM_FIELDS = {}


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("preset,n_prisms,seed", [("medium", 6, 202), ("paper_scale", 20, 302)])
def test_prisms_full_field(gf, orc, preset, n_prisms, seed, prec, tol):
    """The prism part of the medium and paper-scale models at every station:
    the oracle integrates each prism as one merged block (its closed form,
    pinned against the cell-by-cell sum), so the whole field costs one
    evaluation per prism and station; all nine components against it."""
    from synth.density import paint_prisms, random_prisms
    g = PRESETS[preset]
    prisms = random_prisms(g.nx, g.ny, g.nz, n_prisms, seed)
    rho = paint_prisms(np.zeros((g.nz, g.ny, g.nx)), prisms)
    key = (preset, n_prisms, seed)
    if key not in _PRISM_FIELDS:
        st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
        note("prism field %s: oracle at all %d stations" % (preset, len(st)))
        want = orc.blocks_at_stations(g, prisms, st)
        _PRISM_FIELDS[key] = want.reshape(g.ny, g.nx, NC).transpose(2, 0, 1).copy()
    want = _PRISM_FIELDS[key]
    note("prism field %s %s: forward" % (preset, prec))
    got = run_forward(gf, g, rho, mask=ALL9, prec=prec)
    for c in range(NC):
        e = rel(got[c], want[c])
        note("prism field %s %s %s rel %.2e" % (preset, prec, NAMES[c], e))
        assert e <= tol, (NAMES[c], e)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_components_vanishing_on_a_single_row_or_column(gf, orc, prec):
    """One column of cells (nx = 1) puts every station on the x-symmetry
    plane of every cell: gx, gxy, gxz vanish identically, and the library
    returns exact zeros; one row (ny = 1) likewise for gy, gxy, gyz.  The
    other components still match the oracle."""
    dt = torch.float64 if prec == "f64" else torch.float32
    tol = TOL64 if prec == "f64" else TOL32
    for g, odd in ((Geometry(1, 40, 5, 20.0, 25.0, 15.0, 7.0), ("gx", "gxy", "gxz")),
                   (Geometry(40, 1, 5, 20.0, 25.0, 15.0, 7.0), ("gy", "gxy", "gyz"))):
        rho = tiny_density(g.nx, g.ny, g.nz, seed=91, block=None)
        got = run_forward(gf, g, rho, mask=ALL9, prec=prec)
        want = orc.forward_grid(g, rho)
        for c, name in enumerate(NAMES):
            if name in odd:
                assert np.count_nonzero(got[c]) == 0, name
            else:
                assert rel(got[c], want[c]) <= tol, (g, name)
