// Kernel table generation (plan time, FP64).
//
// K_{c,n}(a,b) is the response at a station of the prism at offset
// (a,b) = (l-p, m-q) in layer n (translation equivalence, eq. 7 / eq. 10),
// per unit density and with unit gravitational constant.  Relative to its
// station the prism spans x in [(a-1/2)dx, (a+1/2)dx], y likewise,
// z in [h + z_n, h + z_{n+1}] (z down), z_n the depth of the top of layer n:
// n dz for the paper's uniform layers, any increasing list for a layered
// (depth-stretched) mesh, each layer keeping its own BTTB block.
//
// Near the station the closed forms of the prism integral are used (eq. 2 for
// gz; the tensor forms follow by integrating (3 x_a x_b - r^2 delta_ab)/r^5;
// gx and gy, which section 2.2.3 states to be BTTB as well, integrate x/r^3
// and y/r^3, whose corner terms are eq. 2's with x (or y) and z exchanged,
// the triple integral being symmetric in its variables).
// They are differences of corner terms that grow with distance while the
// result shrinks, so in FP64 they lose digits far away.  Beyond 8
// half-diagonals the cell is integrated instead with a tensor Gauss-Legendre
// rule of the point kernel, whose error falls geometrically with distance;
// the rule shrinks from 6^3 (below 24 half-diagonals) to 4^3 (below 80) to
// 3^3 points as the cell recedes, keeping every entry within ~1e-13 of the
// exact integral.
//
// Values are written straight into the Py x Px circulant embedding (the
// virtual grids of section 2.2.2): offset a at column a mod Px, b at row
// b mod Py, the slots of unreachable offsets left at zero.  One thread
// computes one offset of the quadrant a, b >= 0 and writes its mirror images
// with the component's parity (the potential-field symmetry of section 2.2):
// gz, gxx, gyy even in a and b; gxy odd in both; gxz and gx odd in a; gyz and
// gy odd in b.
#include <hip/hip_runtime.h>

#include "gf_launch.h"

namespace gf {

// Component codes (the bit positions of the public component mask); code 6,
// gzz, is never generated: it is -(gxx + gyy).
enum { K_GZ = 0, K_GXX = 1, K_GXY = 2, K_GXZ = 3, K_GYY = 4, K_GYZ = 5, K_GX = 7, K_GY = 8, NK = 9 };

// Corner term of each closed form.  Cell faces sit at half-integer offsets,
// so a corner is never on x = 0 or y = 0, and z > 0.
__device__ __forceinline__ void corner(double x, double y, double z, double f[NK])
{
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double r = sqrt(x2 + y2 + z2);
    const double ay = asinh(y / sqrt(x2 + z2));
    const double ax = asinh(x / sqrt(y2 + z2));
    const double az = asinh(z / sqrt(x2 + y2));
    const double tz = atan((x * y) / (z * r));
    f[K_GZ] = -(x * ay + y * ax - z * tz);
    f[K_GXX] = -atan2(y * z, x * r);
    f[K_GYY] = -atan2(x * z, y * r);
    f[K_GXY] = log(z + r);
    f[K_GXZ] = ay;
    f[K_GYZ] = ax;
    f[6] = 0.0;
    f[K_GX] = -(z * ay + y * az - x * atan((y * z) / (x * r)));
    f[K_GY] = -(x * az + z * ax - y * atan((x * z) / (y * r)));
}

__device__ void prism_closed(double x1, double x2, double y1, double y2, double z1, double z2,
                             double k[NK])
{
    const double xs[2] = {x1, x2}, ys[2] = {y1, y2}, zs[2] = {z1, z2};
#pragma unroll
    for (int c = 0; c < NK; ++c) k[c] = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double f[NK];
                corner(xs[i], ys[j], zs[q], f);
                // +1 when an odd number of upper bounds (inclusion-exclusion)
                const double mu = ((i + j + q) & 1) ? 1.0 : -1.0;
#pragma unroll
                for (int c = 0; c < NK; ++c) k[c] += mu * f[c];
            }
}

template <int ORD>
__device__ void prism_gauss(double cx, double cy, double cz, double hx, double hy, double hz,
                            const double *gx, const double *gw, double k[NK])
{
    double s[NK] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < ORD; ++i) {
        const double x = cx + hx * gx[i];
#pragma unroll
        for (int j = 0; j < ORD; ++j) {
            const double y = cy + hy * gx[j];
            const double wij = gw[i] * gw[j];
            double t[NK] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < ORD; ++q) {
                const double z = cz + hz * gx[q];
                const double r2 = x * x + y * y + z * z;
                const double ir = rsqrt(r2);
                const double ir3 = ir * ir * ir;
                const double ir5 = ir3 * ir * ir;
                const double w = gw[q];
                t[K_GZ] += w * z * ir3;
                t[K_GXX] += w * (3.0 * x * x - r2) * ir5;
                t[K_GYY] += w * (3.0 * y * y - r2) * ir5;
                t[K_GXY] += w * 3.0 * x * y * ir5;
                t[K_GXZ] += w * 3.0 * x * z * ir5;
                t[K_GYZ] += w * 3.0 * y * z * ir5;
                t[K_GX] += w * x * ir3;
                t[K_GY] += w * y * ir3;
            }
#pragma unroll
            for (int c = 0; c < NK; ++c) s[c] += wij * t[c];
        }
    }
    const double vol = hx * hy * hz;
#pragma unroll
    for (int c = 0; c < NK; ++c) k[c] = s[c] * vol;
}

__global__ void __launch_bounds__(256)
    kgen_field_kernel(double *__restrict__ E, int nl, int n0, int Cs, int4 codes_lo, int2 codes_hi,
                      KgenGeom g, GLRules gl)
{
    const long per_layer = (long)g.nx * g.ny;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per_layer * nl) return;
    const int nloc = (int)(idx / per_layer);
    const long rem = idx % per_layer;
    const int a = (int)(rem % g.nx);
    const int b = (int)(rem / g.nx);
    const int n = n0 + nloc;

    const double x1 = (a - 0.5) * g.dx, x2 = (a + 0.5) * g.dx;
    const double y1 = (b - 0.5) * g.dy, y2 = (b + 0.5) * g.dy;
    const double z1 = g.h + g.zedge[n], z2 = g.h + g.zedge[n + 1];
    const double cx = a * g.dx, cy = b * g.dy, cz = 0.5 * (z1 + z2);
    const double hx = 0.5 * g.dx, hy = 0.5 * g.dy, hz = 0.5 * (z2 - z1);
    const double hd = sqrt(hx * hx + hy * hy + hz * hz);
    const double t = sqrt(cx * cx + cy * cy + cz * cz) / hd;

    double k[NK];
    if (t < g.t_analytic)
        prism_closed(x1, x2, y1, y2, z1, z2, k);
    else if (t < g.t_gl6)
        prism_gauss<6>(cx, cy, cz, hx, hy, hz, gl.x, gl.w, k);
    else if (t < g.t_gl4)
        prism_gauss<4>(cx, cy, cz, hx, hy, hz, gl.x + 6, gl.w + 6, k);
    else
        prism_gauss<3>(cx, cy, cz, hx, hy, hz, gl.x + 10, gl.w + 10, k);

    const int codes[6] = {codes_lo.x, codes_lo.y, codes_lo.z, codes_lo.w, codes_hi.x, codes_hi.y};
    const long field = (long)g.py * g.px;
    const int am = (g.px - a) % g.px, bm = (g.py - b) % g.py;
    for (int c = 0; c < Cs; ++c) {
        const int code = codes[c];
        const int sx = (code == K_GXY || code == K_GXZ || code == K_GX) ? -1 : 1;
        const int sy = (code == K_GXY || code == K_GYZ || code == K_GY) ? -1 : 1;
        double v = k[code];
        // odd components vanish on their symmetry plane
        if ((sx < 0 && a == 0) || (sy < 0 && b == 0)) v = 0.0;
        double *F = E + ((long)nloc * Cs + c) * field;
        F[(long)b * g.px + a] = v;
        F[(long)b * g.px + am] = sx * v;
        F[(long)bm * g.px + a] = sy * v;
        F[(long)bm * g.px + am] = sx * sy * v;
    }
}

int launch_kgen_field(void *E, int nl, int n0, int Cs, const int *codes, const KgenGeom &g,
                      const GLRules &gl, hipStream_t st)
{
    if (Cs < 1 || Cs > 6) return -2;
    int cc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < Cs; ++i) {
        if (codes[i] < 0 || codes[i] >= NK || codes[i] == 6) return -2;
        cc[i] = codes[i];
    }
    const long total = (long)g.nx * g.ny * nl;
    if (total == 0) return 0;
    const long nblk = (total + 255) / 256;
    hipLaunchKernelGGL(kgen_field_kernel, dim3((unsigned)nblk), dim3(256), 0, st, (double *)E, nl, n0,
                       Cs, make_int4(cc[0], cc[1], cc[2], cc[3]), make_int2(cc[4], cc[5]), g, gl);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gf
