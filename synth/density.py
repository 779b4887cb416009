"""Seeded density models (kg/m^3, layout [nz][ny][nx], x fastest).

Recipes:

* ``tiny_density``: uniform(-0.5, 0.5) g/cm^3 plus a +1.0 g/cm^3 block.
* ``prisms_and_grf``: random buried prisms (contrast +-0.2..1.0 g/cm^3,
  5..40 cells per axis) plus a Gaussian random field (sigma 0.05 g/cm^3,
  correlation length 8 cells).
* ``batch_density``: a batch of tiny-style models, one seed per model.
* ``paper_e1_density``: the 300 m cube of section 3.1, 0.3e3 kg/m^3.

All draws use numpy's PCG64 ``default_rng`` so that every consumer sees the
same bits.
"""

import numpy as np
from scipy import ndimage

GCC_TO_SI = 1000.0  # g/cm^3 -> kg/m^3


def tiny_density(nx=16, ny=16, nz=8, seed=101, block=((6, 10), (6, 10), (2, 5)),
                 dtype=np.float64):
    """Uniform(-0.5, 0.5) g/cm^3 plus a +1.0 g/cm^3 block at
    l in [x0,x1), m in [y0,y1), n in [z0,z1)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(-0.5, 0.5, size=(nz, ny, nx))
    if block is not None:
        (x0, x1), (y0, y1), (z0, z1) = block
        rho[z0:z1, y0:y1, x0:x1] += 1.0
    return (rho * GCC_TO_SI).astype(dtype)


def random_prisms(nx, ny, nz, n_prisms, seed, size_range=(5, 40), contrast=(0.2, 1.0)):
    """List of prisms ``(l0, l1, m0, m1, n0, n1, rho_kg_m3)``; each lies fully
    inside the grid, below the top layer, with a random sign."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_prisms):
        sx = int(rng.integers(size_range[0], size_range[1] + 1))
        sy = int(rng.integers(size_range[0], size_range[1] + 1))
        sz = int(rng.integers(size_range[0], size_range[1] + 1))
        sx, sy = min(sx, nx), min(sy, ny)
        sz = max(1, min(sz, nz - 1))
        l0 = int(rng.integers(0, nx - sx + 1))
        m0 = int(rng.integers(0, ny - sy + 1))
        n0 = int(rng.integers(1, nz - sz + 1)) if nz > 1 else 0
        sign = 1.0 if rng.random() < 0.5 else -1.0
        val = sign * rng.uniform(*contrast) * GCC_TO_SI
        out.append((l0, l0 + sx, m0, m0 + sy, n0, n0 + sz, float(val)))
    return out


def gaussian_random_field(nx, ny, nz, seed, sigma=0.05, ell=8.0):
    """Zero-mean Gaussian random field with Gaussian covariance
    exp(-r^2 / (2 ell^2)) (r, ell in cells), rescaled to sample standard
    deviation ``sigma`` g/cm^3; returned in kg/m^3.

    White noise is smoothed by a separable Gaussian filter of width
    ell/sqrt(2) (the square root of the target covariance), reflecting at the
    grid edges.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(size=(nz, ny, nx))
    f = ndimage.gaussian_filter(w, sigma=ell / np.sqrt(2.0), mode="reflect", truncate=4.0)
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f *= sigma / sd
    return f * GCC_TO_SI


def paint_prisms(rho, prisms):
    for (l0, l1, m0, m1, n0, n1, val) in prisms:
        rho[n0:n1, m0:m1, l0:l1] += val
    return rho


def prisms_and_grf(nx, ny, nz, n_prisms, seed_prisms, seed_grf, sigma=0.05, ell=8.0,
                   dtype=np.float64, return_parts=False):
    """Random prisms plus a Gaussian random field.  With ``return_parts`` the
    prism list and the field are returned separately as well."""
    prisms = random_prisms(nx, ny, nz, n_prisms, seed_prisms)
    grf = gaussian_random_field(nx, ny, nz, seed_grf, sigma, ell)
    rho = paint_prisms(grf.copy(), prisms).astype(dtype)
    if return_parts:
        return rho, prisms, grf
    return rho


def batch_density(nb, nx, ny, nz, seed0=400, dtype=np.float64):
    """``nb`` models: uniform(-0.5,0.5) g/cm^3 plus a 4x4x3 +1.0 block at a
    seeded random buried position (seed ``seed0 + b`` for model b)."""
    out = np.empty((nb, nz, ny, nx), dtype=dtype)
    for b in range(nb):
        rng = np.random.default_rng(seed0 + b)
        rho = rng.uniform(-0.5, 0.5, size=(nz, ny, nx))
        bx, by, bz = min(4, nx), min(4, ny), min(3, nz)
        l0 = int(rng.integers(0, nx - bx + 1))
        m0 = int(rng.integers(0, ny - by + 1))
        n0 = int(rng.integers(min(1, nz - bz), nz - bz + 1))
        rho[n0:n0 + bz, m0:m0 + by, l0:l0 + bx] += 1.0
        out[b] = rho * GCC_TO_SI
    return out


def paper_e1_density(dtype=np.float64):
    """Section 3.1: a 300 m cube, top at 500 m, bottom at 800 m, excess
    density 0.3e3 kg/m^3, centred under the origin of a 40x40x20 grid of 50 m
    cells spanning x, y in [-1000, 1000] m; it fills cells 17..22 in x and y
    and layers 10..15."""
    rho = np.zeros((20, 40, 40), dtype=dtype)
    rho[10:16, 17:23, 17:23] = 300.0
    return rho


def sample_stations(nx, ny, n_random, seed):
    """Corners, edge midpoints, the centre and ``n_random`` seeded stations,
    as an int array of (p, q) pairs without duplicates."""
    fixed = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1),
             (nx // 2, 0), (nx // 2, ny - 1), (0, ny // 2), (nx - 1, ny // 2),
             (nx // 2, ny // 2)]
    rng = np.random.default_rng(seed)
    pts = list(dict.fromkeys(fixed))
    seen = set(pts)
    while len(pts) < len(fixed) + n_random and len(seen) < nx * ny:
        p = (int(rng.integers(0, nx)), int(rng.integers(0, ny)))
        if p not in seen:
            seen.add(p)
            pts.append(p)
    return np.array(pts, dtype=np.int32)


def sample_cells(nx, ny, nz, n_random, seed):
    """Grid corners in every axis plus ``n_random`` seeded cells, as an int
    array of (l, m, n) triples without duplicates."""
    fixed = [(l, m, n) for l in (0, nx - 1) for m in (0, ny - 1) for n in (0, nz - 1)]
    fixed.append((nx // 2, ny // 2, nz // 2))
    rng = np.random.default_rng(seed)
    pts = list(dict.fromkeys(fixed))
    seen = set(pts)
    while len(pts) < len(fixed) + n_random and len(seen) < nx * ny * nz:
        c = (int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)))
        if c not in seen:
            seen.add(c)
            pts.append(c)
    return np.array(pts, dtype=np.int32)
