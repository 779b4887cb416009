"""Grid geometries of the workloads (no arithmetic of the method here).

A geometry is the paper's prism discretisation (section 2.1): ``nx*ny*nz``
right rectangular cells of size ``dx*dy*dz``, the model top at depth 0 with
z pointing down, and one station above each surface cell, at the cell-centre
(x, y) and a height ``h`` above the top.
"""

from dataclasses import dataclass, asdict


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    h: float

    @property
    def nd(self) -> int:
        """Number of stations, N_d = nx*ny (section 2.1)."""
        return self.nx * self.ny

    @property
    def nm(self) -> int:
        """Number of cells, N_m = nx*ny*nz (section 2.1)."""
        return self.nx * self.ny * self.nz

    def as_dict(self):
        return asdict(self)


# The five workloads: a tiny grid the oracle sums in full, a medium grid,
# the paper-scale 1024^2 x 100 grid, the inversion-step grid with 32 models
# and the grid sizes of the served request mix.
PRESETS = {
    "tiny": Geometry(16, 16, 8, 50.0, 50.0, 50.0, 25.0),
    "medium": Geometry(256, 256, 64, 25.0, 25.0, 20.0, 10.0),
    "paper_scale": Geometry(1024, 1024, 100, 20.0, 20.0, 20.0, 10.0),
    "inversion": Geometry(512, 512, 128, 20.0, 20.0, 20.0, 10.0),
}

SERVING_N = (64, 128, 256, 512)
SERVING_NZ = (16, 32, 64, 128)


def paper_e1_geometry() -> Geometry:
    """Validation model of section 3.1: 40x40 stations at 50 m spacing, 50 m
    above ground, 40x40x20 cells of 50 m (the cell count 32000 fixes nz=20)."""
    return Geometry(40, 40, 20, 50.0, 50.0, 50.0, 50.0)
