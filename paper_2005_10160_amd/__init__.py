"""MI355X-native fast forward operator for gravity and gravity-gradient data.

The operator of the paper (eq. 3-4, section 2.2): the kernel matrix of each
model layer is a BTTB block (translation equivalence), embedded in a
(2ny x 2nx) circulant whose spectrum stays resident on the GPU, so
d = G rho and g = G^T r are computed by 2-D FFTs and a per-frequency sum
over layers without ever forming G.  The arithmetic is hand-written HIP for
gfx950 in ``libgravfft.so`` behind the C ABI of ``include/gravfft.h``.
"""

from .operator import (
    ALL6,
    ALL7,
    ALL9,
    COMPONENTS,
    GXX,
    GXY,
    GX,
    GXZ,
    GY,
    GYY,
    GYZ,
    GZ,
    GZZ,
    GravityForward,
    GravityOperator,
    Plan,
    adjoint,
    components_mask,
    forward,
    plan,
    plan_layered,
    plan_levels,
    storage_counts,
)

__all__ = [
    "ALL6", "ALL7", "ALL9", "COMPONENTS", "GZ", "GXX", "GXY", "GXZ", "GYY", "GYZ", "GZZ", "GX", "GY",
    "GravityForward", "GravityOperator", "Plan", "adjoint", "components_mask",
    "forward", "plan", "plan_layered", "plan_levels", "storage_counts",
]
