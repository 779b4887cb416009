"""Pins of the CPU oracle against facts outside itself (no GPU).

Each test ties the oracle to mathematics or to the paper rather than to a
retyped copy of its own formulas:
  * Gauss-Legendre brute force of the point kernel (independent integration);
  * the point-mass far-field limit and its convergence order;
  * the trace-free identity (eq. 1 discussion) and tensor symmetry;
  * finite differences of gz, gx and gy in the station position;
  * superposition of cells against one merged prism, and the Bouguer slab;
  * the dense-matrix structure claims (eq. 7, eq. 15-17, BTTB);
  * numpy's FFT applied to the oracle's kernel table (eq. 18);
  * the adjoint dot-product identity;
  * the section 3.1 validation model.
"""

import numpy as np
import pytest

from synth import Geometry, tiny_density, paper_e1_geometry, paper_e1_density

GZ, GXX, GXY, GXZ, GYY, GYZ, GZZ, GX, GY = range(9)
TENSOR = [GXX, GXY, GXZ, GYY, GYZ, GZZ]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- pin 1 ----
def test_gl_rule_matches_library(orc):
    for n in (2, 3, 4, 6, 8, 12, 16):
        x, w = orc.gl_rule(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        order = np.argsort(x)
        assert np.allclose(x[order], xr, rtol=0, atol=1e-15)
        assert np.allclose(w[order], wr, rtol=0, atol=1e-15)


def _random_boxes(seed, count):
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(count):
        sx, sy, sz = rng.uniform(5, 80, size=3)
        cx, cy = rng.uniform(-300, 300, size=2)
        top = rng.uniform(3, 200)
        boxes.append((cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2, top, top + sz))
    # station above the interior of a prism, at its edge, and far away
    boxes.append((-30.0, 50.0, -20.0, 40.0, 5.0, 60.0))
    boxes.append((0.0, 40.0, -40.0, 0.0, 10.0, 30.0))
    boxes.append((2000.0, 2025.0, -1500.0, -1480.0, 100.0, 125.0))
    return boxes


def cancellation_factor(box):
    """The closed forms are differences of corner terms that cancel down to
    ~V/R^3 of their size: their rounding grows as (R/s)^3 (R = centre
    distance, s = half-diagonal).  Returned relative to 24 half-diagonals."""
    c = np.array([(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2])
    s = np.linalg.norm([box[1] - box[0], box[3] - box[2], box[5] - box[4]]) / 2
    return max(1.0, (np.linalg.norm(c) / s / 24.0) ** 3)


def test_closed_form_matches_gauss_legendre(orc):
    """Every component, sign and corner convention against brute-force
    quadrature of G (a/r^3 for gx, gy, gz; (3ab - r^2 delta)/r^5)."""
    for box in _random_boxes(11, 40):
        k = orc.prism(*box)
        q = orc.prism_gl(*box, ratio=0.2, order=10)
        tol = 1e-12 * cancellation_factor(box)
        scale_t = np.abs(k[TENSOR]).max()
        scale_g = np.abs(k[[GZ, GX, GY]]).max()
        assert abs(k[GZ] - q[GZ]) <= tol * abs(q[GZ]), box
        assert np.all(np.abs(k[TENSOR] - q[TENSOR]) <= tol * scale_t), (box, k, q)
        assert np.all(np.abs(k[[GX, GY]] - q[[GX, GY]]) <= tol * scale_g), (box, k, q)


# ---------------------------------------------------------------- pin 2 ----
def _point(G, m, x, y, z):
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    return np.array([
        G * m * z / r ** 3,
        G * m * (3 * x * x - r2) / r ** 5,
        G * m * 3 * x * y / r ** 5,
        G * m * 3 * x * z / r ** 5,
        G * m * (3 * y * y - r2) / r ** 5,
        G * m * 3 * y * z / r ** 5,
        G * m * (3 * z * z - r2) / r ** 5,
        G * m * x / r ** 3,
        G * m * y / r ** 3,
    ])


@pytest.mark.parametrize("sides,slope", [((10.0, 10.0, 10.0), -4.0), ((10.0, 6.0, 14.0), -2.0)])
def test_far_field_point_mass_limit(orc, sides, slope):
    """A prism far away acts as a point mass G m k(R); the relative error
    falls as (a/R)^4 for a cube (no quadrupole) and as (a/R)^2 otherwise.
    This fixes the sign, the constant, the units and the axis convention."""
    G = orc.grav_const()
    assert G == 6.672e-11  # the constant printed with eq. 2
    ax, ay, az = sides
    direction = np.array([0.37, -0.52, 0.77])
    direction /= np.linalg.norm(direction)
    Rs = np.geomspace(10 * ax, 300 * ax, 8)
    errs = []
    for R in Rs:
        cx, cy, cz = R * direction
        k = orc.prism(cx - ax / 2, cx + ax / 2, cy - ay / 2, cy + ay / 2, cz - az / 2, cz + az / 2)
        p = _point(G, ax * ay * az, cx, cy, cz)
        assert np.sign(k[GZ]) == 1.0
        assert (np.sign(k[GX]), np.sign(k[GY])) == (np.sign(cx), np.sign(cy))
        errs.append(np.linalg.norm(k - p) / np.linalg.norm(p))
    fit = np.polyfit(np.log(Rs), np.log(errs), 1)[0]
    assert abs(fit - slope) < 0.2, (fit, errs)


# ---------------------------------------------------------------- pin 3 ----
def test_trace_free_per_prism(orc):
    for box in _random_boxes(12, 60):
        k = orc.prism(*box)
        scale = max(abs(k[GXX]), abs(k[GYY]), abs(k[GZZ]))
        assert abs(k[GXX] + k[GYY] + k[GZZ]) <= 1e-14 * scale * cancellation_factor(box)


def test_trace_free_total_field(orc):
    g = Geometry(9, 7, 4, 30.0, 40.0, 25.0, 15.0)
    rho = tiny_density(9, 7, 4, seed=5, block=None)
    d = orc.forward_grid(g, rho)
    scale = np.abs(d[[GXX, GYY, GZZ]]).max()
    assert np.abs(d[GXX] + d[GYY] + d[GZZ]).max() <= 1e-13 * scale


# ---------------------------------------------------------------- pin 4 ----
def test_symmetry_and_parity_of_offset_table(orc):
    """Section 2.2: the field is symmetric about the X and Y axes.  gz, gxx,
    gyy are even in a and b; gxy is odd in both; gxz and gx odd in a, even in
    b; gyz and gy the reverse; swapping x and y (dx = dy) swaps gxx<->gyy,
    gxz<->gyz, gx<->gy."""
    g = Geometry(12, 12, 3, 20.0, 20.0, 15.0, 7.0)
    for n in range(g.nz):
        t = orc.kernel_table(g, n)           # [c][b][a]
        fa = t[:, :, ::-1]                   # a -> -a
        fb = t[:, ::-1, :]                   # b -> -b
        for c, (sa, sb) in {GZ: (1, 1), GXX: (1, 1), GYY: (1, 1), GZZ: (1, 1),
                            GXY: (-1, -1), GXZ: (-1, 1), GYZ: (1, -1), GX: (-1, 1), GY: (1, -1)}.items():
            s = np.abs(t[c]).max()
            assert np.abs(fa[c] - sa * t[c]).max() <= 4e-16 * s, c
            assert np.abs(fb[c] - sb * t[c]).max() <= 4e-16 * s, c
        tr = t.transpose(0, 2, 1)            # a <-> b
        for c1, c2 in ((GXX, GYY), (GXZ, GYZ), (GZ, GZ), (GXY, GXY), (GZZ, GZZ), (GX, GY)):
            s = np.abs(t[c1]).max()
            assert np.abs(tr[c2] - t[c1]).max() <= 4e-16 * s, (c1, c2)


# ---------------------------------------------------------------- pin 5 ----
def test_tensor_is_derivative_of_gz(orc):
    """Central differences in the station position: d gz/dx0 = gxz,
    d gz/dy0 = gyz, d gz/dz0 = gzz, d gx/dx0 = gxx, d gx/dy0 = d gy/dx0 =
    gxy, d gx/dz0 = gxz, d gy/dy0 = gyy, d gy/dz0 = gyz, d gxz/dx0 =
    d gxx/dz0, d gxz/dy0 = d gxy/dz0, d gyz/dy0 = d gyy/dz0.  Moving the
    station by +e moves the relative (source - station) bounds by -e."""
    for box in _random_boxes(13, 12):
        x1, x2, y1, y2, z1, z2 = box
        e = 1e-4 * z1  # truncation ~ (e / nearest distance)^2

        def k(dx=0.0, dy=0.0, dz=0.0):
            return orc.prism(x1 - dx, x2 - dx, y1 - dy, y2 - dy, z1 - dz, z2 - dz)

        dX = (k(dx=e) - k(dx=-e)) / (2 * e)
        dY = (k(dy=e) - k(dy=-e)) / (2 * e)
        dZ = (k(dz=e) - k(dz=-e)) / (2 * e)
        k0 = k()
        st = np.abs(k0[TENSOR]).max()
        for got, want in ((dX[GZ], k0[GXZ]), (dY[GZ], k0[GYZ]), (dZ[GZ], k0[GZZ]),
                          (dX[GX], k0[GXX]), (dY[GX], k0[GXY]), (dZ[GX], k0[GXZ]),
                          (dX[GY], k0[GXY]), (dY[GY], k0[GYY]), (dZ[GY], k0[GYZ])):
            assert abs(got - want) <= 1e-6 * st, (box, got, want)
        s3 = max(np.abs(dX[TENSOR]).max(), np.abs(dY[TENSOR]).max(), np.abs(dZ[TENSOR]).max())
        for got, want in ((dX[GXZ], dZ[GXX]), (dY[GXZ], dZ[GXY]), (dY[GYZ], dZ[GYY]),
                          (dX[GXY], dY[GXX]), (dY[GXY], dX[GYY])):
            assert abs(got - want) <= 1e-6 * s3, (box, got, want)


# ---------------------------------------------------------------- pin 6 ----
def test_cells_sum_to_merged_prism(orc):
    """Superposition (eq. 3): the direct sum over the cells of a uniform block
    equals one closed-form evaluation of the merged block."""
    g = Geometry(14, 11, 6, 25.0, 30.0, 20.0, 12.0)
    blocks = [(2, 9, 3, 8, 1, 4, 800.0), (10, 14, 0, 5, 3, 6, -350.0), (0, 14, 0, 11, 0, 1, 120.0)]
    rho = np.zeros((g.nz, g.ny, g.nx))
    for (l0, l1, m0, m1, n0, n1, v) in blocks:
        rho[n0:n1, m0:m1, l0:l1] += v
    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    want = orc.blocks_at_stations(g, blocks, st)
    got = orc.forward(g, rho, st)
    for c in range(orc.NCOMP):
        assert rel(got[:, c], want[:, c]) <= 1e-12, c


# ---------------------------------------------------------------- pin 7 ----
def test_bouguer_slab_limit(orc):
    """A uniform slab of thickness t: gz -> 2 pi G rho t at its centre as the
    slab widens, and the vertical gradient there -> 0."""
    G = orc.grav_const()
    rho, t, top = 1000.0, 100.0, 50.0
    want = 2 * np.pi * G * rho * t
    prev_err, prev_gzz = None, None
    for W in (1e3, 1e4, 1e5, 1e6):
        k = orc.prism(-W, W, -W, W, top, top + t) * rho
        err = abs(k[GZ] - want) / want
        if prev_err is not None:
            assert err < prev_err / 5
            assert abs(k[GZZ]) < abs(prev_gzz) / 5
        prev_err, prev_gzz = err, k[GZZ]
    assert prev_err < 1e-4


# ---------------------------------------------------------------- pin 8 ----
def test_dense_matrix_structure(orc):
    """Eq. 7: entries depend only on (l-p, m-q, n).  Eq. 15-17: equal
    diagonals along x.  BTTB: equal blocks along block diagonals in y.  The
    dense matrix is built from absolute positions; the offset table from
    offsets alone."""
    g = Geometry(5, 4, 3, 20.0, 30.0, 25.0, 10.0)
    for comp in (GZ, GXY, GXZ, GYZ, GX, GY):
        Gm = orc.dense_matrix(g, comp)                      # [i][j]
        G5 = Gm.reshape(g.ny, g.nx, g.nz, g.ny, g.nx)       # [q][p][n][m][l]
        s = np.abs(Gm).max()
        tables = [orc.kernel_table(g, n)[comp] for n in range(g.nz)]
        for q in range(g.ny):
            for p in range(g.nx):
                for n in range(g.nz):
                    want = tables[n][(np.arange(g.ny) - q + g.ny - 1)[:, None],
                                     (np.arange(g.nx) - p + g.nx - 1)[None, :]]
                    assert np.abs(G5[q, p, n] - want).max() <= 1e-14 * s
        # Toeplitz along x inside each block, block-Toeplitz along y
        assert np.abs(G5[:, 1:, :, :, 1:] - G5[:, :-1, :, :, :-1]).max() <= 1e-14 * s
        assert np.abs(G5[1:, :, :, 1:, :] - G5[:-1, :, :, :-1, :]).max() <= 1e-14 * s


# ---------------------------------------------------------------- pin 9 ----
def fft_from_tables(g, rho, tables, px, py):
    """Library-FFT form of eq. 18 on the oracle's tables: each layer's table is
    placed circularly on a Py x Px grid (offset a at index a mod Px); the
    density is zero-padded; d = IDFT2(conj(DFT2(K)) DFT2(rho))[:ny,:nx]."""
    out = np.zeros((len(tables[0]), g.ny, g.nx))
    a = np.arange(-(g.nx - 1), g.nx) % px
    b = np.arange(-(g.ny - 1), g.ny) % py
    for n in range(g.nz):
        rp = np.zeros((py, px))
        rp[:g.ny, :g.nx] = rho[n]
        rh = np.fft.fft2(rp)
        for c in range(len(tables[n])):
            emb = np.zeros((py, px))
            emb[np.ix_(b, a)] = tables[n][c]
            out[c] += np.real(np.fft.ifft2(np.conj(np.fft.fft2(emb)) * rh))[:g.ny, :g.nx]
    return out


@pytest.mark.parametrize("geom,pad", [
    (Geometry(16, 16, 8, 50.0, 50.0, 50.0, 25.0), (0, 0)),
    (Geometry(12, 20, 5, 20.0, 30.0, 10.0, 8.0), (0, 0)),
    (Geometry(12, 20, 5, 20.0, 30.0, 10.0, 8.0), (7, 3)),
])
def test_circulant_embedding_equals_direct_sum(orc, geom, pad):
    rho = tiny_density(geom.nx, geom.ny, geom.nz, seed=101,
                       block=((3, 7), (4, 9), (1, 3)))
    tables = [orc.kernel_table(geom, n) for n in range(geom.nz)]
    px, py = 2 * geom.nx + pad[0], 2 * geom.ny + pad[1]
    got = fft_from_tables(geom, rho, tables, px, py)
    want = orc.forward_grid(geom, rho)
    for c in range(orc.NCOMP):
        assert rel(got[c], want[c]) <= 1e-14, c


# --------------------------------------------------------------- pin 10 ----
def test_adjoint_dot_product_and_dense_transpose(orc):
    g = Geometry(6, 5, 3, 20.0, 25.0, 15.0, 9.0)
    rng = np.random.default_rng(7)
    m = rng.standard_normal((g.nz, g.ny, g.nx)) * 500
    r = rng.standard_normal((orc.NCOMP, g.ny, g.nx))
    comps = [GZ, GXX, GXY, GXZ, GYY, GYZ, GX, GY]  # every independent component
    mask = sum(1 << c for c in comps)
    d = orc.forward_grid(g, m)
    lhs = sum(np.vdot(d[c], r[c]) for c in comps)
    gt = orc.adjoint(g, r, mask)
    rhs = np.vdot(m, gt)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(d[comps]) * np.linalg.norm(r[comps])
    want = sum(orc.dense_matrix(g, c).T @ r[c].ravel() for c in comps)
    assert rel(gt.ravel(), want) <= 1e-14
    # cells listed one by one give the same numbers
    cells = np.array([(1, 2, 0), (5, 4, 2), (0, 0, 1)])
    sub = orc.adjoint(g, r, mask, cells)
    for i, (l, m_, n) in enumerate(cells):
        assert sub[i] == gt[n, m_, l]


def test_batch_forward_matches_single(orc):
    g = Geometry(7, 6, 3, 20.0, 20.0, 20.0, 10.0)
    rho = np.stack([tiny_density(7, 6, 3, seed=s, block=None) for s in (1, 2, 3)])
    st = np.array([(0, 0), (6, 5), (3, 2)])
    both = orc.forward(g, rho, st)
    for b in range(3):
        assert np.array_equal(both[b], orc.forward(g, rho[b], st))


# --------------------------------------------------------------- pin 12 ----
def _read_fixture(path):
    vals = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    return vals


def test_paper_validation_model(orc):
    """Section 3.1: a 300 m cube (top 500 m, bottom 800 m, 0.3e3 kg/m^3) under
    a 40x40 grid of stations 50 m apart and 50 m up.  The fast (circulant)
    result differs from the plain one by ~13 orders of magnitude less than
    the field; here the library-FFT form of the oracle tables, the cell-by-cell
    direct sum and the merged-prism closed form are compared."""
    import os
    fx = _read_fixture(os.path.join(os.path.dirname(__file__), "golden", "paper_e1_model.txt"))
    g = paper_e1_geometry()
    rho = paper_e1_density()
    assert (g.nx, g.ny, g.nz) == tuple(int(v[0]) for v in (fx["nx"], fx["ny"], fx["nz"]))
    assert g.nd == fx["n_stations"][0] and g.nm == fx["n_cells"][0]
    assert g.dx == fx["station_spacing_m"][0] and g.h == fx["station_height_m"][0]
    cells = np.argwhere(rho > 0)
    assert rho.max() == fx["density_contrast_kg_m3"][0]
    assert (cells[:, 0].min() * g.dz, (cells[:, 0].max() + 1) * g.dz) == (
        fx["body_top_depth_m"][0], fx["body_bottom_depth_m"][0])
    assert (cells[:, 2].max() + 1 - cells[:, 2].min()) * g.dx == fx["body_size_m"][0]
    # the body is centred under the grid centre
    assert (cells[:, 2].min() + cells[:, 2].max() + 1) * g.dx / 2 == g.nx * g.dx / 2

    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    merged = orc.blocks_at_stations(g, [(17, 23, 17, 23, 10, 16, 300.0)], st)
    merged = merged.reshape(g.ny, g.nx, orc.NCOMP).transpose(2, 0, 1)
    tables = [orc.kernel_table(g, n) for n in range(10, 16)]
    sub = Geometry(g.nx, g.ny, 6, g.dx, g.dy, g.dz, g.h + 10 * g.dz)
    fast = fft_from_tables(sub, rho[10:16], [orc.kernel_table(sub, n) for n in range(6)],
                           2 * g.nx, 2 * g.ny)
    for c in range(orc.NCOMP):  # Fig. 6-7 include the first derivatives gx, gy
        assert rel(fast[c], merged[c]) <= 10.0 ** -fx["residual_orders"][0], c
    # the layered tables equal the shifted-geometry tables (same prisms)
    for n in range(6):
        assert np.allclose(tables[n], orc.kernel_table(sub, n), rtol=1e-15, atol=0)
    # a sample of stations by the plain cell-by-cell sum
    some = st[::97]
    direct = orc.forward(g, rho, some)
    for i, (p, q) in enumerate(some):
        assert np.allclose(direct[i], merged[:, q, p], rtol=1e-12, atol=1e-12 * np.abs(merged).max())


# --------------------------------------------------------------- pin 13 ----
def test_layered_mesh_merges_uniform_layers(orc):
    """Layers of unequal thickness (a depth-stretched mesh): a layer spanning
    two uniform layers acts as both of them with the same density
    (superposition, eq. 3), forward and adjoint.  The merged layer's closed
    form uses other corners than the two thin layers', so this checks the
    layered path against the pinned uniform one."""
    g5 = Geometry(9, 7, 5, 30.0, 40.0, 15.0, 12.0)
    thick = [2, 1, 2]                              # uniform layers per merged layer
    edges = np.concatenate([[0.0], np.cumsum(thick) * g5.dz])
    g3 = Geometry(g5.nx, g5.ny, 3, g5.dx, g5.dy, 99.0, g5.h)   # dz unused with edges
    rho3 = tiny_density(g3.nx, g3.ny, 3, seed=31, block=None)
    rho5 = np.repeat(rho3, thick, axis=0)
    got = orc.forward_grid(g3, rho3, zedges=edges)
    want = orc.forward_grid(g5, rho5)
    for c in range(orc.NCOMP):
        assert rel(got[c], want[c]) <= 1e-13, c
    rng = np.random.default_rng(32)
    r = rng.standard_normal((orc.NCOMP, g5.ny, g5.nx))
    a3 = orc.adjoint(g3, r, 0x1FF, zedges=edges)
    a5 = orc.adjoint(g5, r, 0x1FF)
    merged = np.add.reduceat(a5, np.concatenate([[0], np.cumsum(thick)[:-1]]), axis=0)
    assert rel(a3, merged) <= 1e-13


def test_layered_mesh_buried_top_and_blocks(orc):
    """A mesh whose top lies at depth z0 below the surface equals the uniform
    mesh seen from stations z0 higher; a stretched mesh's cells sum to the
    merged prisms of its blocks; bad edge lists are refused."""
    g = Geometry(8, 6, 4, 25.0, 20.0, 10.0, 6.0)
    z0 = 37.0
    edges = z0 + g.dz * np.arange(g.nz + 1)
    rho = tiny_density(g.nx, g.ny, g.nz, seed=33, block=None)
    got = orc.forward_grid(g, rho, zedges=edges)
    high = Geometry(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h + z0)
    want = orc.forward_grid(high, rho)
    for c in range(orc.NCOMP):
        assert rel(got[c], want[c]) <= 1e-13, c

    gs = Geometry(14, 11, 6, 25.0, 30.0, 1.0, 12.0)
    es = np.concatenate([[0.0], np.cumsum(8.0 * 1.3 ** np.arange(6))])
    blocks = [(2, 9, 3, 8, 1, 4, 800.0), (10, 14, 0, 5, 3, 6, -350.0), (0, 14, 0, 11, 0, 1, 120.0)]
    rho = np.zeros((gs.nz, gs.ny, gs.nx))
    for (l0, l1, m0, m1, n0, n1, v) in blocks:
        rho[n0:n1, m0:m1, l0:l1] += v
    st = np.array([(p, q) for q in range(gs.ny) for p in range(gs.nx)])
    want = orc.blocks_at_stations(gs, blocks, st, zedges=es)
    got = orc.forward(gs, rho, st, zedges=es)
    for c in range(orc.NCOMP):
        assert rel(got[:, c], want[:, c]) <= 1e-12, c

    for bad in ([0.0, 10.0, 10.0, 30.0, 40.0], [-1.0, 10.0, 20.0, 30.0, 40.0],
                [0.0, 10.0, np.nan, 30.0, 40.0]):
        with pytest.raises(ValueError):
            orc.forward_grid(g, rho[:4, :6, :8], zedges=bad)


def test_layered_offset_table_is_a_shifted_uniform_layer(orc):
    """The offset table of layer n of a stretched mesh equals layer 0 of a
    uniform mesh whose top is z_n deeper and whose layers are z_{n+1} - z_n
    thick: the same prisms (eq. 7 per layer), in both table modes."""
    g = Geometry(9, 6, 5, 20.0, 30.0, 1.0, 7.0)
    z = np.concatenate([[3.0], 3.0 + np.cumsum(4.0 * 1.6 ** np.arange(g.nz))])
    for n in range(g.nz):
        u = Geometry(g.nx, g.ny, 1, g.dx, g.dy, z[n + 1] - z[n], g.h + z[n])
        for mode in (0, 1):
            got = orc.kernel_table(g, n, mode=mode, zedges=z)
            want = orc.kernel_table(u, 0, mode=mode)
            for c in range(orc.NCOMP):
                s = np.abs(want[c]).max()
                assert np.abs(got[c] - want[c]).max() <= 1e-14 * s, (n, mode, c)


# --------------------------------------------------------------- pin 14 ----
def test_levels_are_translation_equivalent_in_depth(orc):
    """Eq. 10 for the equal-dimension survey: with station levels dz apart,
    the block of level t and layer n is the block of level 0 and layer
    n + t (the same prism seen from the same relative position)."""
    g = Geometry(9, 7, 6, 20.0, 30.0, 15.0, 7.0)
    for t in (1, 2, 5):
        gt = Geometry(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h + t * g.dz)
        for n in range(g.nz - t):
            a = orc.kernel_table(gt, n)
            b = orc.kernel_table(g, n + t)
            for c in range(orc.NCOMP):
                s = np.abs(b[c]).max()
                assert np.abs(a[c] - b[c]).max() <= 1e-14 * s, (t, n, c)


def test_levels_forward_and_adjoint_compose(orc):
    """The multi-level operator stacks the single-plane operators of each
    level, and its adjoint sums theirs: the dot-product identity over all
    levels and components."""
    g = Geometry(6, 5, 3, 20.0, 25.0, 15.0, 9.0)
    levels = 4
    rng = np.random.default_rng(61)
    m = rng.standard_normal((g.nz, g.ny, g.nx)) * 300
    d = orc.forward_levels(g, m, levels)                       # (levels, nst, NCOMP)
    assert d.shape == (levels, g.nx * g.ny, orc.NCOMP)
    r = rng.standard_normal((levels, orc.NCOMP, g.ny, g.nx))
    comps = [0, 1, 2, 3, 4, 5, 7, 8]
    mask = sum(1 << c for c in comps)
    gt = orc.adjoint_levels(g, r, mask, levels)
    dg = d.reshape(levels, g.ny, g.nx, orc.NCOMP).transpose(0, 3, 1, 2)
    lhs = sum(np.vdot(dg[t, c], r[t, c]) for t in range(levels) for c in comps)
    rhs = np.vdot(m, gt)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(dg[:, comps]) * np.linalg.norm(r[:, comps])
    # level 0 is the single plane
    assert np.array_equal(d[0], orc.forward(g, m))


def test_fp64_build_of_the_oracle(orc):
    """The oracle's plain-double build (timed beside the long-double one) is
    the same computation: it agrees to 1e-12 on the tiny grid, and on a wide
    grid, where the closed forms' corner terms cancel over many orders, to
    the 1e-8 its rounding allows (the long-double build is the reference)."""
    g = Geometry(16, 16, 8, 50.0, 50.0, 50.0, 25.0)
    rho = tiny_density(g.nx, g.ny, g.nz)
    a = orc.forward(g, rho)
    b = orc.forward_fp64(g, rho)
    for c in range(orc.NCOMP):
        assert rel(b[:, c], a[:, c]) <= 1e-12, c
    w = Geometry(512, 512, 2, 20.0, 20.0, 20.0, 10.0)
    rho = np.random.default_rng(3).uniform(-500, 500, size=(w.nz, w.ny, w.nx))
    st = np.array([(0, 0), (256, 256)])
    a = orc.forward(w, rho, st)
    b = orc.forward_fp64(w, rho, st)
    for c in range(orc.NCOMP):
        assert rel(b[:, c], a[:, c]) <= 1e-8, c


# --------------------------------------------------------------- pin 15 ----
def _cell_box(g, a, b, n):
    """Bounds of the cell at offset (a, b) in layer n relative to its station
    (source minus station, z down): the geometry of section 2.1 with the
    stations above the cell centres."""
    return ((a - 0.5) * g.dx, (a + 0.5) * g.dx, (b - 0.5) * g.dy, (b + 0.5) * g.dy,
            g.h + n * g.dz, g.h + (n + 1) * g.dz)


def _offsets_in_shell(g, n, lo, hi, count, seed):
    """Offsets (a, b) of layer n whose cell centre lies between lo and hi
    half-diagonals from the station."""
    rng = np.random.default_rng(seed)
    s = np.sqrt(g.dx ** 2 + g.dy ** 2 + g.dz ** 2) / 2
    zc = g.h + (n + 0.5) * g.dz
    out = []
    while len(out) < count:
        dist = rng.uniform(lo, hi) * s
        if dist <= zc:
            continue
        rxy = np.sqrt(dist ** 2 - zc ** 2)
        phi = rng.uniform(0, 2 * np.pi)
        a, b = int(round(rxy * np.cos(phi) / g.dx)), int(round(rxy * np.sin(phi) / g.dy))
        c = np.sqrt((a * g.dx) ** 2 + (b * g.dy) ** 2 + zc ** 2) / s
        if lo <= c <= hi:
            out.append((a, b))
    return np.array(out)


def test_far_field_rule_of_the_offset_table(orc):
    """The offset table's far-field branch (mode 1: one 8^3 Gauss-Legendre
    rule over the cell beyond 24 half-diagonals) against two routes that do
    not share it: the closed form (mode 0) from 24 to 100 half-diagonals,
    where its cancellation still leaves ~1e-11, and an adaptive brute force
    of another order and subdivision from 100 to 1000 half-diagonals."""
    g = Geometry(1, 1, 6, 20.0, 30.0, 15.0, 10.0)
    for n in (0, 3, 5):
        ab = _offsets_in_shell(g, n, 24.0, 100.0, 40, seed=80 + n)
        k1 = orc.offset_kernels(g, n, ab[:, 0], ab[:, 1], mode=1)
        k0 = orc.offset_kernels(g, n, ab[:, 0], ab[:, 1], mode=0)
        for i, (a, b) in enumerate(ab):
            box = _cell_box(g, a, b, n)
            tol = 1e-12 * cancellation_factor(box)
            st = np.abs(k0[i][TENSOR]).max()
            sg = np.abs(k0[i][[GZ, GX, GY]]).max()
            assert np.all(np.abs(k1[i][TENSOR] - k0[i][TENSOR]) <= tol * st), (n, a, b)
            assert np.all(np.abs(k1[i][[GZ, GX, GY]] - k0[i][[GZ, GX, GY]]) <= tol * sg), (n, a, b)
        ab = _offsets_in_shell(g, n, 100.0, 1000.0, 12, seed=90 + n)
        k1 = orc.offset_kernels(g, n, ab[:, 0], ab[:, 1], mode=1)
        for i, (a, b) in enumerate(ab):
            q = orc.prism_gl(*_cell_box(g, a, b, n), ratio=0.004, order=5)
            st = np.abs(q[TENSOR]).max()
            sg = np.abs(q[[GZ, GX, GY]]).max()
            assert np.all(np.abs(k1[i][TENSOR] - q[TENSOR]) <= 1e-14 * st), (n, a, b)
            assert np.all(np.abs(k1[i][[GZ, GX, GY]] - q[[GZ, GX, GY]]) <= 1e-14 * sg), (n, a, b)
    # the full table switches branch inside it; both halves agree with mode 0
    # where the closed form is still exact to its cancellation
    gw = Geometry(40, 30, 2, 20.0, 30.0, 15.0, 10.0)
    for n in range(gw.nz):
        t1 = orc.kernel_table(gw, n, mode=1)
        t0 = orc.kernel_table(gw, n, mode=0)
        for c in range(orc.NCOMP):
            s = np.abs(t0[c]).max()
            assert np.abs(t1[c] - t0[c]).max() <= 1e-12 * s, (n, c)


def test_levels_are_the_model_under_empty_layers(orc):
    """Level t of the equal-dimension survey (stations t dz higher) is the
    single-plane operator of a grid with t empty layers on top of the model,
    forward and adjoint (superposition, eq. 3: empty cells add nothing).
    dx, dy and dz all differ, so a level spacing taken from the wrong axis
    fails here."""
    g = Geometry(6, 5, 3, 20.0, 25.0, 15.0, 9.0)
    levels = 4
    rng = np.random.default_rng(63)
    m = rng.standard_normal((g.nz, g.ny, g.nx)) * 300
    d = orc.forward_levels(g, m, levels)                       # (levels, nst, NCOMP)
    r = rng.standard_normal((levels, orc.NCOMP, g.ny, g.nx))
    mask = 0x1BF                                               # all but gzz
    gt = orc.adjoint_levels(g, r, mask, levels)
    total = np.zeros_like(gt)
    for t in range(levels):
        big = Geometry(g.nx, g.ny, g.nz + t, g.dx, g.dy, g.dz, g.h)
        mb = np.concatenate([np.zeros((t, g.ny, g.nx)), m])
        want = orc.forward(big, mb)
        for c in range(orc.NCOMP):
            assert rel(d[t][:, c], want[:, c]) <= 1e-13, (t, c)
        total += orc.adjoint(big, r[t], mask)[t:]
    assert rel(gt, total) <= 1e-13


def test_tabulated_sum_equals_direct_sum(orc):
    """The tabulated direct sum (each layer's offset table built once, then
    multiply-adds) is the same sum as the cell-by-cell one: equal within
    rounding on grids with nx != ny, on a layered mesh, for a batch and for
    a subset of the components (the others are returned as zero)."""
    g = Geometry(14, 11, 6, 25.0, 30.0, 20.0, 12.0)
    rho = np.stack([tiny_density(g.nx, g.ny, g.nz, seed=s, block=None) for s in (4, 5)])
    st = np.array([(p, q) for q in range(g.ny) for p in range(g.nx)])
    want = orc.forward(g, rho, st)
    got = orc.forward_tabulated(g, rho, st, mask=0x1FF)
    for c in range(orc.NCOMP):
        assert rel(got[..., c], want[..., c]) <= 1e-14, c
    z = np.concatenate([[4.0], 4.0 + np.cumsum(6.0 * 1.4 ** np.arange(g.nz))])
    want = orc.forward(g, rho[0], st[::7], zedges=z)
    got = orc.forward_tabulated(g, rho[0], st[::7], mask=0x89, zedges=z)  # gz, gxz, gx
    for c in range(orc.NCOMP):
        if 0x89 >> c & 1:
            assert rel(got[:, c], want[:, c]) <= 1e-14, c
        else:
            assert not got[:, c].any(), c
    w = Geometry(37, 5, 2, 20.0, 15.0, 10.0, 3.0)     # a row length that is not a multiple of 4
    rho = tiny_density(w.nx, w.ny, w.nz, seed=6, block=None)
    st = np.array([(0, 0), (36, 4), (18, 2), (5, 3)])
    assert rel(orc.forward_tabulated(w, rho, st, mask=0x3F)[:, :6], orc.forward(w, rho, st)[:, :6]) <= 1e-14
