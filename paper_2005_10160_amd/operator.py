"""Python face of the fast gravity / gravity-gradient operator.

``plan(nx, ny, nz, dx, dy, dz, h, components)`` builds the resident kernel
spectra on the GPU; ``forward(plan, rho, d)`` computes d = G rho (eq. 4) and
``adjoint(plan, r, g)`` computes g = G^T r.  PyTorch supplies device memory
and the stream; every arithmetic step runs in ``libgravfft.so``.
"""

import ctypes

import torch

from . import _native as nat

COMPONENTS = ("gz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "gx", "gy")
GZ, GXX, GXY, GXZ, GYY, GYZ, GZZ, GX, GY = (1 << i for i in range(9))
ALL6 = 0x3F
ALL7 = 0x7F
ALL9 = 0x1FF


def components_mask(components):
    """Accept a bit mask or an iterable of component names."""
    if isinstance(components, int):
        return components
    m = 0
    for c in components:
        m |= 1 << COMPONENTS.index(c)
    return m


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A geometry's resident kernel spectra (see include/gravfft.h)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, h, components=ALL6, precision="f64",
                 max_batch=0, device=None, stream=None, zedges=None, levels=1):
        lib = nat.load()
        device = torch.device("cuda") if device is None else torch.device(device)
        if device.type != "cuda":
            raise ValueError("the operator runs on a GPU device, got %s" % device)
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = device
        prec = {"f64": nat.GF_F64, "fp64": nat.GF_F64, "float64": nat.GF_F64,
                "f32": nat.GF_F32, "fp32": nat.GF_F32, "float32": nat.GF_F32}[str(precision).lower()]
        self.precision = "f64" if prec == nat.GF_F64 else "f32"
        self.dtype = torch.float64 if prec == nat.GF_F64 else torch.float32
        self.mask = components_mask(components)
        self.geometry = (int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(h))
        self.zedges = None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _stream_handle(stream)
            if zedges is not None and int(levels) != 1:
                raise ValueError("observation levels need uniform layers")
            if int(levels) != 1:
                nat.check(lib.gf_plan_create_levels(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                                                    float(h), int(levels), ctypes.c_uint(self.mask), prec,
                                                    int(max_batch), st, ctypes.byref(handle)),
                          "gf_plan_create_levels")
            elif zedges is None:
                nat.check(lib.gf_plan_create(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(h),
                                             ctypes.c_uint(self.mask), prec, int(max_batch), st,
                                             ctypes.byref(handle)),
                          "gf_plan_create")
            else:
                z = (ctypes.c_double * len(zedges))(*[float(v) for v in zedges])
                if len(zedges) != int(nz) + 1:
                    raise ValueError("zedges must hold nz + 1 depths, got %d" % len(zedges))
                nat.check(lib.gf_plan_create_layered(int(nx), int(ny), int(nz), float(dx), float(dy), z, float(h),
                                                     ctypes.c_uint(self.mask), prec, int(max_batch), st,
                                                     ctypes.byref(handle)),
                          "gf_plan_create_layered")
                self.zedges = tuple(float(v) for v in zedges)
        self._h = handle
        info = nat.PlanInfo()
        nat.check(lib.gf_plan_get_info(self._h, ctypes.byref(info)), "gf_plan_get_info")
        self.info = info
        self.nx, self.ny, self.nz = info.nx, info.ny, info.nz
        self.n_out = info.n_out
        self.n_levels = info.n_levels
        self.col_groups = info.col_groups
        self.level_path = info.level_path
        self.level_chunk = info.level_chunk
        # one data plane per observation level
        self.data_shape = ((self.n_levels,) if self.n_levels > 1 else ()) + (self.n_out, self.ny, self.nx)
        self.out_components = tuple(COMPONENTS[i] for i in range(len(COMPONENTS)) if self.mask >> i & 1)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            nat.load().gf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- facts ----------------------------------------------------------------
    @property
    def spectra_bytes(self):
        return int(self.info.spectra_bytes)

    @property
    def plan_ms(self):
        return float(self.info.plan_ms)

    def storage(self):
        """The paper's stored-kernel counts for this geometry beside what the
        plan keeps resident.  The counts are per component and are scaled by
        the resident spectral components and the element size into bytes;
        `resident_bytes` is the device memory the plan holds for its spectra
        (one real per frequency of the quarter plane, rows padded to the
        column pass's pitch, plus the depth-transformed spectra of a levels
        plan that transforms in depth)."""
        i = self.info
        c = storage_counts(i.nx, i.ny, i.nz, i.n_levels)
        elem = 8 if self.precision == "f64" else 4
        out = {k: c[k] for k in ("dense", "ega", "ega_virtual", "bttb")}
        out["ratio"] = c["ratio"]
        out["components"] = int(i.n_spec)
        out["element_bytes"] = elem
        for k in ("dense", "bttb"):
            out[k + "_bytes"] = c[k] * i.n_spec * elem
        out["quarter_plane_per_layer"] = (i.px // 2 + 1) * (i.py // 2 + 1)
        out["resident_bytes"] = int(i.spectra_bytes)
        out["resident_over_bttb"] = int(i.spectra_bytes) / (c["bttb"] * i.n_spec * elem)
        return out

    def workspace_bytes(self, op, batch):
        out = ctypes.c_size_t()
        opc = nat.GF_OP_FORWARD if op in ("forward", 0) else nat.GF_OP_ADJOINT
        nat.check(nat.load().gf_workspace_bytes(self._h, opc, int(batch), ctypes.byref(out)), "gf_workspace_bytes")
        return int(out.value)

    def _workspace(self, op, batch, workspace, stream=None):
        need = self.workspace_bytes(op, batch)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        if workspace.device != self.device or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous tensor on %s" % self.device)
        nbytes = workspace.numel() * workspace.element_size()
        if stream is not None:
            # the caching allocator must not hand this memory out before the
            # kernels on `stream` are done with it
            workspace.record_stream(stream)
        return workspace, nbytes

    def _check_in(self, x, shape_tail, name):
        if not isinstance(x, torch.Tensor) or x.device != self.device:
            raise ValueError("%s must be a tensor on %s" % (name, self.device))
        if x.dtype != self.dtype:
            raise ValueError("%s must be %s for a %s plan" % (name, self.dtype, self.precision))
        if not x.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if x.dim() == len(shape_tail):
            x = x.unsqueeze(0)
        if tuple(x.shape[1:]) != tuple(shape_tail) or x.dim() != len(shape_tail) + 1:
            raise ValueError("%s has shape %s, expected [B]+%s" % (name, tuple(x.shape), list(shape_tail)))
        return x

    # -- operator ----------------------------------------------------------
    def forward(self, rho, out=None, workspace=None, stream=None):
        """d = G rho.  rho [B][nz][ny][nx] (or [nz][ny][nx]) -> d [B][C][ny][nx]
        ([B][levels][C][ny][nx] for a plan of several observation levels)."""
        squeeze = rho.dim() == 3
        rho = self._check_in(rho, (self.nz, self.ny, self.nx), "rho")
        B = rho.shape[0]
        if out is None:
            out = torch.empty((B,) + self.data_shape, dtype=self.dtype, device=self.device)
        out = self._check_in(out, self.data_shape, "d")
        if out.shape[0] != B:
            raise ValueError("d batch %d != rho batch %d" % (out.shape[0], B))
        ws, nb = self._workspace("forward", B, workspace, stream)
        with torch.cuda.device(self.device):
            nat.check(nat.load().gf_forward(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            B, ctypes.c_void_p(ws.data_ptr()), nb, _stream_handle(stream)),
                      "gf_forward")
        return out[0] if squeeze else out

    def adjoint(self, r, out=None, workspace=None, stream=None):
        """g = G^T r.  r [B][C][ny][nx] (or [C][ny][nx]; with levels
        [B][levels][C][ny][nx]) -> g [B][nz][ny][nx]."""
        squeeze = r.dim() == len(self.data_shape)
        r = self._check_in(r, self.data_shape, "r")
        B = r.shape[0]
        if out is None:
            out = torch.empty((B, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        out = self._check_in(out, (self.nz, self.ny, self.nx), "g")
        if out.shape[0] != B:
            raise ValueError("g batch %d != r batch %d" % (out.shape[0], B))
        ws, nb = self._workspace("adjoint", B, workspace, stream)
        with torch.cuda.device(self.device):
            nat.check(nat.load().gf_adjoint(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            B, ctypes.c_void_p(ws.data_ptr()), nb, _stream_handle(stream)),
                      "gf_adjoint")
        return out[0] if squeeze else out

    # -- timing ----------------------------------------------------------------
    def set_timing(self, enable=True):
        nat.check(nat.load().gf_plan_set_timing(self._h, 1 if enable else 0), "gf_plan_set_timing")

    def last_pass_ms(self, op="forward"):
        """(row transform, column pass, inverse row transform) ms of the last
        timed call of op."""
        ms = (ctypes.c_double * 3)()
        opc = nat.GF_OP_FORWARD if op in ("forward", 0) else nat.GF_OP_ADJOINT
        nat.check(nat.load().gf_plan_last_pass_ms(self._h, opc, ms), "gf_plan_last_pass_ms")
        return tuple(ms)

    # -- test access ---------------------------------------------------------
    def debug_kernel_table(self, n):
        import numpy as np
        out = np.zeros((len(COMPONENTS), 2 * self.ny - 1, 2 * self.nx - 1))
        nat.check(nat.load().gf_debug_kernel_table(self._h, int(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                  "gf_debug_kernel_table")
        return out

    def debug_spectrum(self, component, n):
        import numpy as np
        bit = components_mask([component]) if isinstance(component, str) else int(component)
        out = np.zeros((self.info.px // 2 + 1, self.info.py // 2 + 1))
        nat.check(nat.load().gf_debug_spectrum(self._h, ctypes.c_uint(bit), int(n),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                  "gf_debug_spectrum")
        return out


def storage_counts(nx, ny, nz, levels=1):
    """Kernel values one component needs stored under each scheme the paper
    compares, for nx x ny stations on `levels` planes over nx x ny x nz cells.

    dense        eq. 5: the whole matrix, N_d x N_m (section 2.1; with several
                 planes N_d counts every station, as in the 1.1e16 figure of
                 section 2.2 for 100 planes over 1024 x 1024 x 100 cells)
    ega          eq. 9: the kernel of the computation origin against every
                 cell, valid through the potential-field symmetry (section 2.2.1)
    ega_virtual  eq. 11: the origin against the cells of the virtual grid,
                 translation only (section 2.2.2)
    bttb         eq. 22: first row and column of every Toeplitz level,
                 (2nx-1)(2ny-1) per layer offset; a plane of stations sees nz
                 offsets, `levels` planes see nz + levels - 1 (n - t + 1 of
                 eq. 10)
    ratio        eq. 20: the BTTB count of one layer block over its dense count
    """
    nx, ny, nz, levels = int(nx), int(ny), int(nz), int(levels)
    nd = nx * ny * levels
    nm = nx * ny * nz
    offsets = nz + levels - 1
    return {
        "dense": nd * nm,
        "ega": nm,
        "ega_virtual": 2 * nx * 2 * ny * 2 * nz,
        "bttb": (2 * nx - 1) * (2 * ny - 1) * offsets,
        "ratio": (2 * nx - 1) / (nx * nx) * (2 * ny - 1) / (ny * ny),
    }


def plan(nx, ny, nz, dx, dy, dz, h, components=ALL6, precision="f64", max_batch=0, device=None, stream=None):
    return Plan(nx, ny, nz, dx, dy, dz, h, components, precision, max_batch, device, stream)


def plan_levels(nx, ny, nz, dx, dy, dz, h, levels, components=ALL6, precision="f64", max_batch=0, device=None,
                stream=None):
    """Plan of the equal-dimension survey: stations on `levels` planes at
    heights h + t dz (t = 0 .. levels-1) above the model top; data
    [B][levels][C][ny][nx]."""
    return Plan(nx, ny, nz, dx, dy, dz, h, components, precision, max_batch, device, stream, levels=levels)


def plan_layered(nx, ny, dx, dy, zedges, h, components=ALL6, precision="f64", max_batch=0, device=None,
                 stream=None):
    """Plan of a layered mesh: layer n spans depths [zedges[n], zedges[n+1]]
    (len(zedges) = nz + 1, strictly increasing, zedges[0] >= 0)."""
    nz = len(zedges) - 1
    return Plan(nx, ny, nz, dx, dy, 0.0, h, components, precision, max_batch, device, stream, zedges=zedges)


def forward(p, rho, d=None, workspace=None, stream=None):
    return p.forward(rho, d, workspace, stream)


def adjoint(p, r, g=None, workspace=None, stream=None):
    return p.adjoint(r, g, workspace, stream)


class GravityForward(torch.autograd.Function):
    """d = G rho with backward grad_rho = G^T grad_d (G is constant)."""

    @staticmethod
    def forward(ctx, rho, p):
        ctx.plan = p
        return p.forward(rho.contiguous())

    @staticmethod
    def backward(ctx, grad_d):
        return ctx.plan.adjoint(grad_d.contiguous()), None


class GravityOperator(torch.nn.Module):
    """nn.Module wrapper: ``GravityOperator(plan)(rho) -> d``, differentiable in rho."""

    def __init__(self, p):
        super().__init__()
        self.plan = p

    def forward(self, rho):
        return GravityForward.apply(rho, self.plan)
