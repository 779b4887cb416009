"""CPU oracle of the prism gravity / gravity-gradient forward operator.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_2005_10160_amd``; the two meet only
through the seeded inputs of ``synth``.

The arithmetic lives in ``gravity_oracle.c`` (plain C, x87 long double,
OpenMP over stations / layers, no FMA contraction); this module only marshals
numpy arrays through ctypes.

Component order everywhere: gz, gxx, gxy, gxz, gyy, gyz, gzz, gx, gy.
"""

import ctypes
import os
import subprocess
import threading

import numpy as np

COMPONENTS = ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "gx", "gy")
NCOMP = 9

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gravity_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_gravity_oracle.so")
_LIB64_PATH = os.path.join(_HERE, "_gravity_oracle_f64.so")
_LIBSAN_PATH = os.path.join(_HERE, "_gravity_oracle_san.so")
_lock = threading.Lock()
_lib = None
_lib64 = None

# Set to "1" (before the first call) to load the build instrumented with the
# address and undefined-behaviour sanitizers instead of the reference build;
# the process must then start with the sanitizer runtime preloaded.
SANITIZE_ENV = "GF_ORACLE_SANITIZE"
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build(force=False, sanitize=False):
    """Compile the oracle with gcc (no fast-math, no FMA contraction): the
    long-double reference and, from the same source, its plain-double build
    (timed beside it, never a reference).  sanitize=True builds only the
    sanitizer-instrumented variant of the reference."""
    opt = ["-O3", "-march=x86-64-v3"]
    builds = ((_LIBSAN_PATH, SANITIZE_FLAGS),) if sanitize else ((_LIB_PATH, opt), (_LIB64_PATH, opt + ["-DORC_FP64"]))
    for path, extra in builds:
        if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(_SRC):
            continue
        tmp = path + ".tmp%d" % os.getpid()
        cmd = (["gcc"] + extra + ["-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
                                  "-o", tmp, _SRC, "-lm"])
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return builds[0][0]


def _load(fp64=False):
    global _lib, _lib64
    with _lock:
        if (_lib64 if fp64 else _lib) is not None:
            return _lib64 if fp64 else _lib
        if os.environ.get(SANITIZE_ENV) == "1" and not fp64:
            lib = ctypes.CDLL(build(sanitize=True))
        else:
            build()
            lib = ctypes.CDLL(_LIB64_PATH if fp64 else _LIB_PATH)
        d, i, u = ctypes.c_double, ctypes.c_int, ctypes.c_uint
        pd = ctypes.POINTER(ctypes.c_double)
        pi = ctypes.POINTER(ctypes.c_int)
        lib.orc_prism.argtypes = [d] * 6 + [pd]
        lib.orc_prism.restype = None
        lib.orc_prism_gl.argtypes = [d] * 6 + [d, i, pd]
        lib.orc_prism_gl.restype = i
        lib.orc_gl_rule.argtypes = [i, pd, pd]
        lib.orc_gl_rule.restype = i
        lib.orc_offset_kernels.argtypes = [d, d, d, d, i, i, pi, pi, i, pd]
        lib.orc_offset_kernels.restype = i
        lib.orc_forward.argtypes = [i, i, i, d, d, d, d, i, pd, i, pi, pi, pd]
        lib.orc_forward.restype = i
        lib.orc_adjoint.argtypes = [i, i, i, d, d, d, d, i, u, pd, i, pi, pi, pi, pd]
        lib.orc_adjoint.restype = i
        lib.orc_dense_matrix.argtypes = [i, i, i, d, d, d, d, i, pd]
        lib.orc_dense_matrix.restype = i
        lib.orc_blocks_at_stations.argtypes = [i, i, i, d, d, d, d, i, pi, pd, i, pi, pi, pd]
        lib.orc_blocks_at_stations.restype = i
        lib.orc_offset_kernels_z.argtypes = [d, d, d, pd, d, i, i, pi, pi, i, pd]
        lib.orc_offset_kernels_z.restype = i
        lib.orc_forward_z.argtypes = [i, i, i, d, d, d, pd, d, i, pd, i, pi, pi, pd]
        lib.orc_forward_z.restype = i
        lib.orc_adjoint_z.argtypes = [i, i, i, d, d, d, pd, d, i, u, pd, i, pi, pi, pi, pd]
        lib.orc_adjoint_z.restype = i
        lib.orc_forward_tab_z.argtypes = [i, i, i, d, d, d, pd, d, i, pd, u, i, pi, pi, pd]
        lib.orc_forward_tab_z.restype = i
        lib.orc_blocks_at_stations_z.argtypes = [i, i, i, d, d, d, pd, d, i, pi, pd, i, pi, pi, pd]
        lib.orc_blocks_at_stations_z.restype = i
        lib.orc_max_threads.restype = i
        lib.orc_set_threads.argtypes = [i]
        lib.orc_grav_const.restype = d
        if fp64:
            _lib64 = lib
        else:
            _lib = lib
        return lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _geom(g):
    return (int(g.nx), int(g.ny), int(g.nz), float(g.dx), float(g.dy), float(g.dz), float(g.h))


def _edges(geom, zedges):
    """Layer edges as a contiguous float64 array of nz + 1 depths (layer n
    spans [zedges[n], zedges[n+1]] below the top), or None for uniform
    layers of thickness geom.dz."""
    if zedges is None:
        return None
    z = np.ascontiguousarray(zedges, dtype=np.float64).ravel()
    if z.size != geom.nz + 1:
        raise ValueError("zedges must hold nz + 1 depths")
    return z


def _geom_z(g, z):
    nx, ny, nz, dx, dy, dz, h = _geom(g)
    return (nx, ny, nz, dx, dy, dz, _pd(z), h)


def grav_const():
    return _load().orc_grav_const()


def max_threads():
    return _load().orc_max_threads()


def set_threads(n):
    _load().orc_set_threads(int(n))


def prism(x1, x2, y1, y2, z1, z2):
    """Kernel of one prism with bounds relative to the station (source minus
    station, z down, 0 < z1 < z2), per kg/m^3, in SI: array of NCOMP."""
    out = np.zeros(NCOMP)
    _load().orc_prism(float(x1), float(x2), float(y1), float(y2), float(z1), float(z2), _pd(out))
    return out


def prism_gl(x1, x2, y1, y2, z1, z2, ratio=0.25, order=8):
    """Adaptive Gauss-Legendre brute force of the point kernel over a prism."""
    out = np.zeros(NCOMP)
    rc = _load().orc_prism_gl(float(x1), float(x2), float(y1), float(y2), float(z1), float(z2),
                              float(ratio), int(order), _pd(out))
    if rc != 0:
        raise ValueError("bad Gauss-Legendre order / ratio")
    return out


def gl_rule(order):
    x = np.zeros(order)
    w = np.zeros(order)
    if _load().orc_gl_rule(int(order), _pd(x), _pd(w)) != 0:
        raise ValueError("bad order")
    return x, w


def offset_kernels(geom, n, a, b, mode=0, zedges=None):
    """Kernel of the cell at offset (a, b) = (l-p, m-q) in layer n relative to
    its station (translation equivalence, eq. 7/10).  mode 0: closed form;
    mode 1: closed form near, 8^3 Gauss-Legendre beyond 24 half-diagonals.
    Returns (len(a), NCOMP)."""
    a = np.ascontiguousarray(a, dtype=np.int32).ravel()
    b = np.ascontiguousarray(b, dtype=np.int32).ravel()
    assert a.shape == b.shape
    out = np.zeros((a.size, NCOMP))
    z = _edges(geom, zedges)
    if z is not None:
        rc = _load().orc_offset_kernels_z(float(geom.dx), float(geom.dy), float(geom.dz), _pd(z), float(geom.h),
                                          int(n), int(a.size), _pi(a), _pi(b), int(mode), _pd(out))
    else:
        rc = _load().orc_offset_kernels(float(geom.dx), float(geom.dy), float(geom.dz), float(geom.h),
                                        int(n), int(a.size), _pi(a), _pi(b), int(mode), _pd(out))
    if rc != 0:
        raise ValueError("bad geometry")
    return out


def kernel_table(geom, n, mode=0, zedges=None):
    """Full offset table of layer n: (NCOMP, 2ny-1, 2nx-1), index [c][b+ny-1][a+nx-1]."""
    aa, bb = np.meshgrid(np.arange(-(geom.nx - 1), geom.nx), np.arange(-(geom.ny - 1), geom.ny))
    k = offset_kernels(geom, n, aa.ravel(), bb.ravel(), mode, zedges)
    return k.T.reshape(NCOMP, 2 * geom.ny - 1, 2 * geom.nx - 1)


def forward_fp64(geom, rho, stations=None):
    """The direct sum of forward() evaluated in plain double (the same code
    built with double arithmetic): reported for timing and for the size of
    its rounding, not used as a reference."""
    return forward(geom, rho, stations, _fp64=True)


def forward(geom, rho, stations=None, zedges=None, _fp64=False):
    """Direct sum d = G rho (eq. 3) at stations (array of (p, q)); all
    stations in row order (q major) when None.  rho: (nz,ny,nx) or
    (nb,nz,ny,nx) in kg/m^3.  zedges: nz + 1 layer-edge depths of a layered
    mesh (None: uniform layers of geom.dz).  Returns (nb, nst, NCOMP) (nb
    dropped for 3-D rho)."""
    rho = np.asarray(rho, dtype=np.float64)
    squeeze = rho.ndim == 3
    if squeeze:
        rho = rho[None]
    nb = rho.shape[0]
    assert rho.shape[1:] == (geom.nz, geom.ny, geom.nx), rho.shape
    rho = np.ascontiguousarray(rho)
    if stations is None:
        qq, pp = np.meshgrid(np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
        stations = np.stack([pp.ravel(), qq.ravel()], axis=1)
    st = np.ascontiguousarray(stations, dtype=np.int32).reshape(-1, 2)
    sp = np.ascontiguousarray(st[:, 0])
    sq = np.ascontiguousarray(st[:, 1])
    out = np.zeros((nb, st.shape[0], NCOMP))
    z = _edges(geom, zedges)
    if _fp64:
        rc = _load(True).orc_forward(*_geom(geom), nb, _pd(rho), int(st.shape[0]), _pi(sp), _pi(sq), _pd(out))
    elif z is not None:
        rc = _load().orc_forward_z(*_geom_z(geom, z), nb, _pd(rho), int(st.shape[0]), _pi(sp), _pi(sq), _pd(out))
    else:
        rc = _load().orc_forward(*_geom(geom), nb, _pd(rho), int(st.shape[0]), _pi(sp), _pi(sq), _pd(out))
    if rc != 0:
        raise ValueError("oracle forward failed (%d)" % rc)
    return out[0] if squeeze else out


def forward_tabulated(geom, rho, stations=None, mask=0x3F, zedges=None):
    """The direct sum of forward() (eq. 3) with each layer's kernel tabulated
    once over all offsets (eq. 7, eq. 10) from the same closed form, then
    summed by multiply-adds in the order: row sums over l, rows in ascending
    m, layers in ascending n, all in long double.  Fast enough for every
    station of a 256^2 x 64 grid or a thousand stations of a 1024^2 x 100
    grid.  mask: components summed (bit c = COMPONENTS[c]); the others are 0.
    Returns (nb, nst, NCOMP) (nb dropped for 3-D rho)."""
    rho = np.asarray(rho, dtype=np.float64)
    squeeze = rho.ndim == 3
    if squeeze:
        rho = rho[None]
    nb = rho.shape[0]
    assert rho.shape[1:] == (geom.nz, geom.ny, geom.nx), rho.shape
    rho = np.ascontiguousarray(rho)
    if stations is None:
        qq, pp = np.meshgrid(np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
        stations = np.stack([pp.ravel(), qq.ravel()], axis=1)
    st = np.ascontiguousarray(stations, dtype=np.int32).reshape(-1, 2)
    sp = np.ascontiguousarray(st[:, 0])
    sq = np.ascontiguousarray(st[:, 1])
    out = np.zeros((nb, st.shape[0], NCOMP))
    z = _edges(geom, zedges)
    zp = ctypes.POINTER(ctypes.c_double)() if z is None else _pd(z)
    nx, ny, nz, dx, dy, dz, h = _geom(geom)
    rc = _load().orc_forward_tab_z(nx, ny, nz, dx, dy, dz, zp, h, nb, _pd(rho), ctypes.c_uint(int(mask)),
                                   int(st.shape[0]), _pi(sp), _pi(sq), _pd(out))
    if rc != 0:
        raise ValueError("oracle tabulated forward failed (%d)" % rc)
    return out[0] if squeeze else out


def forward_grid(geom, rho, zedges=None):
    """Direct sum at every station: (nb, NCOMP, ny, nx) (nb dropped for 3-D rho)."""
    squeeze = np.asarray(rho).ndim == 3
    out = forward(geom, rho, zedges=zedges)
    if squeeze:
        out = out[None]
    nb = out.shape[0]
    res = out.reshape(nb, geom.ny, geom.nx, NCOMP).transpose(0, 3, 1, 2).copy()
    return res[0] if squeeze else res


def adjoint(geom, r, mask, cells=None, zedges=None):
    """Direct adjoint g(l,m,n) = sum_c sum_{p,q} G_c[(p,q),(l,m,n)] r_c(p,q).
    r: (NCOMP, ny, nx) or (nb, NCOMP, ny, nx) indexed by component slot; only slots in
    ``mask`` (bit c = component c) are read.  cells: array of (l, m, n);
    every cell when None (returned as (nb, nz, ny, nx))."""
    r = np.asarray(r, dtype=np.float64)
    squeeze = r.ndim == 3
    if squeeze:
        r = r[None]
    nb = r.shape[0]
    assert r.shape[1:] == (NCOMP, geom.ny, geom.nx), r.shape
    r = np.ascontiguousarray(r)
    full = cells is None
    if full:
        nn, mm, ll = np.meshgrid(np.arange(geom.nz), np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
        cells = np.stack([ll.ravel(), mm.ravel(), nn.ravel()], axis=1)
    cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
    cl, cm, cn = (np.ascontiguousarray(cells[:, i]) for i in range(3))
    out = np.zeros((nb, cells.shape[0]))
    z = _edges(geom, zedges)
    if z is not None:
        rc = _load().orc_adjoint_z(*_geom_z(geom, z), nb, ctypes.c_uint(int(mask)), _pd(r), int(cells.shape[0]),
                                   _pi(cl), _pi(cm), _pi(cn), _pd(out))
    else:
        rc = _load().orc_adjoint(*_geom(geom), nb, ctypes.c_uint(int(mask)), _pd(r), int(cells.shape[0]),
                                 _pi(cl), _pi(cm), _pi(cn), _pd(out))
    if rc != 0:
        raise ValueError("oracle adjoint failed (%d)" % rc)
    if full:
        out = out.reshape(nb, geom.nz, geom.ny, geom.nx)
    return out[0] if squeeze else out


def dense_matrix(geom, comp):
    """Dense kernel matrix (Nd x Nm) of component ``comp`` (index into
    COMPONENTS): station i = p + q nx, cell j = l + m nx + n nx ny (eq. 12)."""
    out = np.zeros((geom.nx * geom.ny, geom.nx * geom.ny * geom.nz))
    rc = _load().orc_dense_matrix(*_geom(geom), int(comp), _pd(out))
    if rc != 0:
        raise ValueError("bad arguments")
    return out


def blocks_at_stations(geom, blocks, stations, zedges=None):
    """Superposition of uniform blocks, each integrated as one merged prism.
    blocks: iterable of (l0, l1, m0, m1, n0, n1, rho).  Returns (nst, NCOMP)."""
    blocks = list(blocks)
    blk = np.ascontiguousarray(np.array([b[:6] for b in blocks], dtype=np.int32).reshape(-1))
    val = np.ascontiguousarray(np.array([b[6] for b in blocks], dtype=np.float64))
    st = np.ascontiguousarray(stations, dtype=np.int32).reshape(-1, 2)
    sp = np.ascontiguousarray(st[:, 0])
    sq = np.ascontiguousarray(st[:, 1])
    out = np.zeros((st.shape[0], NCOMP))
    z = _edges(geom, zedges)
    if z is not None:
        rc = _load().orc_blocks_at_stations_z(*_geom_z(geom, z), len(blocks), _pi(blk), _pd(val),
                                              int(st.shape[0]), _pi(sp), _pi(sq), _pd(out))
    else:
        rc = _load().orc_blocks_at_stations(*_geom(geom), len(blocks), _pi(blk), _pd(val), int(st.shape[0]),
                                            _pi(sp), _pi(sq), _pd(out))
    if rc != 0:
        raise ValueError("bad blocks")
    return out


class _AtHeight:
    """The geometry `geom` with its station plane at height `h`."""

    def __init__(self, geom, h):
        self.nx, self.ny, self.nz = geom.nx, geom.ny, geom.nz
        self.dx, self.dy, self.dz = geom.dx, geom.dy, geom.dz
        self.h = h


def forward_levels(geom, rho, levels, stations=None):
    """Equal-dimension survey (section 2.2, Fig. 2a): stations on `levels`
    planes at heights h + t dz, t = 0 .. levels-1, above the model top; each
    level is the direct sum (eq. 3) of its own plane.  Returns
    (nb, levels, nst, NCOMP) (nb dropped for 3-D rho)."""
    out = [forward(_AtHeight(geom, geom.h + t * geom.dz), rho, stations) for t in range(levels)]
    return np.stack(out, axis=-3)


def adjoint_levels(geom, r, mask, levels, cells=None):
    """Adjoint of forward_levels: sum over levels of each plane's adjoint.
    r: (levels, NCOMP, ny, nx) or (nb, levels, NCOMP, ny, nx)."""
    r = np.asarray(r, dtype=np.float64)
    lev_axis = r.ndim - 4
    total = None
    for t in range(levels):
        rt = np.ascontiguousarray(np.take(r, t, axis=lev_axis))
        a = adjoint(_AtHeight(geom, geom.h + t * geom.dz), rt, mask, cells)
        total = a if total is None else total + a
    return total
