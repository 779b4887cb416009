/*
 * CPU oracle for the prism gravity / gravity-gradient forward operator.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the product path never does.  It
 * shares no code with the HIP implementation.
 *
 * What it computes is the plain definition of the operator:
 *
 *   d_c(p,q) = sum_{l,m,n} G_c[(p,q),(l,m,n)] rho(l,m,n)      (eq. 3 / eq. 4)
 *
 * where G_c is the exact volume integral of the point-source kernel over the
 * right rectangular prism of cell (l,m,n), for component c.  Evaluation is in
 * x87 extended precision (long double, 64-bit mantissa): the closed forms below
 * are differences of eight corner terms that grow with distance while the
 * result shrinks, so plain double loses up to ~1e-10 relative on the deep
 * layers of a 1024^2 grid; extended precision keeps the oracle ~2000x below
 * that.
 *
 * Conventions (the paper leaves them implicit, section 2.1):
 *   - z points down; the model top is z = 0; the station plane is z = -h.
 *   - Cell (l,m,n) spans x in [l dx,(l+1)dx], y in [m dy,(m+1)dy],
 *     z in [n dz,(n+1)dz]; station (p,q) sits at ((p+1/2)dx, (q+1/2)dy, -h),
 *     one above each surface cell (section 2.1: N_d = nx*ny).
 *   - Layered meshes (the *_z entry points): layer n spans depths
 *     [zedge[n], zedge[n+1]] instead, for a strictly increasing zedge[nz+1]
 *     with zedge[0] >= 0.  The paper takes the layers uniform (section 2.1);
 *     translation equivalence (eq. 7) holds within each layer whatever its
 *     thickness, so each layer keeps its own BTTB block.
 *   - Relative coordinates are source minus station, so z > 0 inside cells.
 *   - U = G rho \iiint dV / r;  g = grad U (pointing at the mass, gz > 0 for
 *     a positive mass below);  T_ab = d^2 U / da db.
 *   - Component order: gz, gxx, gxy, gxz, gyy, gyz, gzz, gx, gy.
 *   - G = 6.672e-11 N m^2 / kg^2, the constant printed with eq. 2.
 *
 * Closed forms, with corners (x_i, y_j, z_k), i,j,k in {lower, upper}, and
 * sign mu = +1 when an odd number of the three coordinates are upper bounds
 * (the inclusion-exclusion of a triple definite integral; eq. 2's
 * mu_ijk = (-1)^(i+j+k) with 1-based bounds):
 *   gz  = -G rho sum mu [ x asinh(y/sqrt(x^2+z^2)) + y asinh(x/sqrt(y^2+z^2))
 *                         - z atan(x y / (z r)) ]                    (eq. 2)
 *   gxx = -G rho sum mu atan2(y z, x r)
 *   gyy = -G rho sum mu atan2(x z, y r)
 *   gzz = -G rho sum mu atan(x y / (z r))
 *   gxy =  G rho sum mu ln(z + r)
 *   gxz =  G rho sum mu asinh(y / sqrt(x^2+z^2))
 *   gyz =  G rho sum mu asinh(x / sqrt(y^2+z^2))
 *   gx  = -G rho sum mu [ z asinh(y/sqrt(x^2+z^2)) + y asinh(z/sqrt(x^2+y^2))
 *                         - x atan(y z / (x r)) ]
 *   gy  = -G rho sum mu [ x asinh(z/sqrt(x^2+y^2)) + z asinh(x/sqrt(y^2+z^2))
 *                         - y atan(x z / (y r)) ]
 * The tensor forms follow from integrating (3 a b - r^2 delta_ab) / r^5 one
 * axis at a time; eq. 2 reads ln(y/sqrt(x^2+z^2) + sqrt(1 + y^2/(x^2+z^2))),
 * which is asinh(y/sqrt(x^2+z^2)) and is evaluated as such (the form
 * ln(y + r) cancels catastrophically for y < 0).  The first derivatives gx
 * and gy (whose kernels section 2.2.3 also states to be BTTB) integrate x/r^3
 * and y/r^3: the triple integral is symmetric in its three variables, so
 * their corner terms are the gz term with x and z (for gx) or y and z (for
 * gy) exchanged.  Corners never lie on x = 0 or y = 0 (cell faces sit at
 * half-integer offsets), and the jump of atan(y z / (x r)) across x = 0 is
 * killed by its factor x.
 */
#include <stdlib.h>
#include <tgmath.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Built twice: in long double (the reference), and with ORC_FP64 in plain
 * double, whose timing is reported beside it (same code, type-generic math). */
#ifdef ORC_FP64
typedef double ld;
#else
typedef long double ld;
#endif

enum { C_GZ = 0, C_GXX = 1, C_GXY = 2, C_GXZ = 3, C_GYY = 4, C_GYZ = 5, C_GZZ = 6, C_GX = 7, C_GY = 8,
       NCOMP = 9 };

static const ld GRAV = (ld)6.672e-11L; /* eq. 2 */

int orc_ncomp(void) { return NCOMP; }
double orc_grav_const(void) { return (double)GRAV; }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Corner terms of the closed forms (without G rho and without mu).          */
/* ------------------------------------------------------------------------ */

static void corner_terms(ld x, ld y, ld z, ld f[NCOMP])
{
    ld x2 = x * x, y2 = y * y, z2 = z * z;
    ld r = sqrt(x2 + y2 + z2);
    ld sxz = sqrt(x2 + z2);
    ld syz = sqrt(y2 + z2);
    ld ash_y = asinh(y / sxz);        /* = ln(y + r) - ln sqrt(x^2+z^2) */
    ld ash_x = asinh(x / syz);        /* = ln(x + r) - ln sqrt(y^2+z^2) */
    /* On a corner at x = y = 0 (a station over a cell edge) the terms
     * y asinh(z/sqrt(x^2+y^2)) and x atan(y z / (x r)) have the limit 0:
     * the factor vanishes while asinh grows like ln(1/|y|) and atan stays
     * bounded. */
    ld sxy = sqrt(x2 + y2);
    ld ash_z = sxy > 0 ? asinh(z / sxy) : 0;   /* only ever multiplied by x or y */
    ld at_x = x != 0 ? atan((y * z) / (x * r)) : 0;
    ld at_y = y != 0 ? atan((x * z) / (y * r)) : 0;
    ld at_z = atan((x * y) / (z * r));
    f[C_GZ] = -(x * ash_y + y * ash_x - z * at_z);
    f[C_GXX] = -atan2(y * z, x * r);
    f[C_GYY] = -atan2(x * z, y * r);
    f[C_GZZ] = -at_z;
    f[C_GXY] = log(z + r);
    f[C_GXZ] = ash_y;
    f[C_GYZ] = ash_x;
    f[C_GX] = -(z * ash_y + y * ash_z - x * at_x);
    f[C_GY] = -(x * ash_z + z * ash_x - y * at_y);
}

/* mu for corner (i,j,k), each 0 = lower bound, 1 = upper bound. */
static ld corner_sign(int i, int j, int k) { return ((i + j + k) & 1) ? (ld)1 : (ld)-1; }

/* Kernel of one prism (per unit density, G included) from its corners. */
static void prism_ld(ld x1, ld x2, ld y1, ld y2, ld z1, ld z2, ld out[NCOMP])
{
    ld xs[2] = {x1, x2}, ys[2] = {y1, y2}, zs[2] = {z1, z2};
    ld acc[NCOMP] = {0};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                ld f[NCOMP];
                corner_terms(xs[i], ys[j], zs[k], f);
                ld mu = corner_sign(i, j, k);
                for (int c = 0; c < NCOMP; ++c) acc[c] += mu * f[c];
            }
    for (int c = 0; c < NCOMP; ++c) out[c] = GRAV * acc[c];
}

/* Public: one prism given by its bounds relative to the station
 * (source minus station, z down, z1 < z2, z1 > 0).  out[9] in SI per kg/m^3. */
void orc_prism(double x1, double x2, double y1, double y2, double z1, double z2, double out[NCOMP])
{
    ld o[NCOMP];
    prism_ld(x1, x2, y1, y2, z1, z2, o);
    for (int c = 0; c < NCOMP; ++c) out[c] = (double)o[c];
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre brute force of the point-source kernel.                    */
/* ------------------------------------------------------------------------ */

/* Nodes and weights on [-1,1]: Newton iteration on P_n from the Chebyshev
 * guess cos(pi (i+3/4)/(n+1/2)), using the three-term recurrence. */
static void gl_rule(int n, ld *x, ld *w)
{
    const ld PI = (ld)3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld t = cos(PI * (i + (ld)0.75) / (n + (ld)0.5));
        ld dp = 1;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = t;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_n(t), p0 = P_{n-1}(t) */
            dp = n * (t * p1 - p0) / (t * t - 1);
            ld dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < (ld)1e-19L) break;
        }
        {
            ld p0 = 1, p1 = t;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1);
        }
        x[i] = t;
        w[i] = 2 / ((1 - t * t) * dp * dp);
    }
}

/* Point-source kernel at relative position (x,y,z) of a unit mass, G included:
 * g_a = G a / r^3, T_ab = G (3 a b - r^2 delta_ab) / r^5. */
static void point_kernel(ld x, ld y, ld z, ld k[NCOMP])
{
    ld r2 = x * x + y * y + z * z;
    ld r = sqrt(r2);
    ld ir3 = 1 / (r2 * r);
    ld ir5 = ir3 / r2;
    k[C_GZ] = GRAV * z * ir3;
    k[C_GXX] = GRAV * (3 * x * x - r2) * ir5;
    k[C_GYY] = GRAV * (3 * y * y - r2) * ir5;
    k[C_GZZ] = GRAV * (3 * z * z - r2) * ir5;
    k[C_GXY] = GRAV * 3 * x * y * ir5;
    k[C_GXZ] = GRAV * 3 * x * z * ir5;
    k[C_GYZ] = GRAV * 3 * y * z * ir5;
    k[C_GX] = GRAV * x * ir3;
    k[C_GY] = GRAV * y * ir3;
}

#define GL_MAX 32

static void gl_box(ld x1, ld x2, ld y1, ld y2, ld z1, ld z2, int n, const ld *gx, const ld *gw,
                   ld acc[NCOMP])
{
    ld cx = (x1 + x2) / 2, hx = (x2 - x1) / 2;
    ld cy = (y1 + y2) / 2, hy = (y2 - y1) / 2;
    ld cz = (z1 + z2) / 2, hz = (z2 - z1) / 2;
    ld s[NCOMP] = {0};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                ld kk[NCOMP];
                point_kernel(cx + hx * gx[i], cy + hy * gx[j], cz + hz * gx[k], kk);
                ld w = gw[i] * gw[j] * gw[k];
                for (int c = 0; c < NCOMP; ++c) s[c] += w * kk[c];
            }
    for (int c = 0; c < NCOMP; ++c) acc[c] += s[c] * hx * hy * hz;
}

static void gl_adaptive(ld x1, ld x2, ld y1, ld y2, ld z1, ld z2, ld ratio, int n, const ld *gx,
                        const ld *gw, int depth, ld acc[NCOMP])
{
    ld cx = (x1 + x2) / 2, cy = (y1 + y2) / 2, cz = (z1 + z2) / 2;
    ld hd = sqrt((x2 - x1) * (x2 - x1) + (y2 - y1) * (y2 - y1) + (z2 - z1) * (z2 - z1)) / 2;
    ld dist = sqrt(cx * cx + cy * cy + cz * cz);
    if (hd <= ratio * dist || depth >= 24) {
        gl_box(x1, x2, y1, y2, z1, z2, n, gx, gw, acc);
        return;
    }
    ld xb[3] = {x1, cx, x2}, yb[3] = {y1, cy, y2}, zb[3] = {z1, cz, z2};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
                gl_adaptive(xb[i], xb[i + 1], yb[j], yb[j + 1], zb[k], zb[k + 1], ratio, n, gx, gw,
                            depth + 1, acc);
}

/* Public: adaptive tensor Gauss-Legendre integral of the point kernel over a
 * prism (relative bounds as in orc_prism).  Boxes are halved along every axis
 * until half-diagonal / centre distance <= ratio, then integrated with an
 * order^3 rule.  Returns 0, or -1 for a bad order. */
int orc_prism_gl(double x1, double x2, double y1, double y2, double z1, double z2, double ratio,
                 int order, double out[NCOMP])
{
    if (order < 1 || order > GL_MAX || !(ratio > 0)) return -1;
    ld gx[GL_MAX], gw[GL_MAX];
    gl_rule(order, gx, gw);
    ld acc[NCOMP] = {0};
    gl_adaptive(x1, x2, y1, y2, z1, z2, ratio, order, gx, gw, 0, acc);
    for (int c = 0; c < NCOMP; ++c) out[c] = (double)acc[c];
    return 0;
}

/* Public: the rule itself, for tests (nodes on [-1,1]). */
int orc_gl_rule(int order, double *x, double *w)
{
    if (order < 1 || order > GL_MAX) return -1;
    ld gx[GL_MAX], gw[GL_MAX];
    gl_rule(order, gx, gw);
    for (int i = 0; i < order; ++i) {
        x[i] = (double)gx[i];
        w[i] = (double)gw[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Kernel by offset (translation equivalence, eq. 7 / eq. 10).               */
/* ------------------------------------------------------------------------ */

/* Depth of the top of layer n (n = nz: the bottom of the model). */
static ld layer_depth(int n, double dz, const double *zedge)
{
    return zedge ? (ld)zedge[n] : (ld)n * dz;
}

/* 0 when zedge is NULL or a strictly increasing list of nz+1 finite depths
 * starting at >= 0. */
static int check_edges(int nz, const double *zedge)
{
    if (!zedge) return 0;
    if (!(zedge[0] >= 0) || !isfinite(zedge[0])) return -1;
    for (int n = 0; n < nz; ++n)
        if (!(zedge[n + 1] > zedge[n]) || !isfinite(zedge[n + 1])) return -1;
    return 0;
}

/* Bounds of the cell at offset (a, b) = (l - p, m - q) in layer n, relative
 * to its station. */
static void cell_bounds(int a, int b, int n, double dx, double dy, double dz, const double *zedge,
                        double h, ld bx[6])
{
    bx[0] = ((ld)a - (ld)0.5) * dx;
    bx[1] = ((ld)a + (ld)0.5) * dx;
    bx[2] = ((ld)b - (ld)0.5) * dy;
    bx[3] = ((ld)b + (ld)0.5) * dy;
    bx[4] = (ld)h + layer_depth(n, dz, zedge);
    bx[5] = (ld)h + layer_depth(n + 1, dz, zedge);
}

/* Public: kernel values of cells given by offsets (a[i], b[i]) in layer n.
 * mode 0: closed form for every entry.
 * mode 1: closed form when the station-to-cell-centre distance is below 24
 *         half-diagonals, otherwise one 8^3 Gauss-Legendre rule over the cell
 *         (at that distance its truncation error is far below long-double
 *         rounding, while the closed form starts to lose digits).
 * out[count][9]. */
int orc_offset_kernels_z(double dx, double dy, double dz, const double *zedge, double h, int n, int count,
                         const int *a, const int *b, int mode, double *out)
{
    if (!(dx > 0 && dy > 0 && (zedge || dz > 0) && h > 0) || n < 0 || count < 0) return -1;
    if (zedge && check_edges(n + 1, zedge) != 0) return -1;
    ld gx[GL_MAX], gw[GL_MAX];
    gl_rule(8, gx, gw);
    ld tz = layer_depth(n + 1, dz, zedge) - layer_depth(n, dz, zedge);
    ld hd = sqrt((ld)dx * dx + (ld)dy * dy + tz * tz) / 2;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < count; ++i) {
        ld bx[6], o[NCOMP];
        cell_bounds(a[i], b[i], n, dx, dy, dz, zedge, h, bx);
        ld cx = (bx[0] + bx[1]) / 2, cy = (bx[2] + bx[3]) / 2, cz = (bx[4] + bx[5]) / 2;
        ld dist = sqrt(cx * cx + cy * cy + cz * cz);
        if (mode == 1 && dist >= 24 * hd) {
            for (int c = 0; c < NCOMP; ++c) o[c] = 0;
            gl_box(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], 8, gx, gw, o);
        } else {
            prism_ld(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], o);
        }
        for (int c = 0; c < NCOMP; ++c) out[(size_t)i * NCOMP + c] = (double)o[c];
    }
    return 0;
}

int orc_offset_kernels(double dx, double dy, double dz, double h, int n, int count, const int *a,
                       const int *b, int mode, double *out)
{
    return orc_offset_kernels_z(dx, dy, dz, NULL, h, n, count, a, b, mode, out);
}

/* ------------------------------------------------------------------------ */
/* Node planes: corner terms on a plane of grid nodes, reused by the cells   */
/* that share them (each cell still sums its own eight corners).             */
/* ------------------------------------------------------------------------ */

/* Fill plane[(jy*(nxn) + ix)*NCOMP + c] with corner_terms at x = (v0 + ix - 1/2) dx,
 * y = (w0 + jy - 1/2) dy, depth z. */
static void fill_plane(ld *plane, int v0, int nxn, int w0, int nyn, double dx, double dy, ld z)
{
    for (int jy = 0; jy < nyn; ++jy) {
        ld y = ((ld)(w0 + jy) - (ld)0.5) * dy;
        for (int ix = 0; ix < nxn; ++ix) {
            ld x = ((ld)(v0 + ix) - (ld)0.5) * dx;
            corner_terms(x, y, z, plane + ((size_t)jy * nxn + ix) * NCOMP);
        }
    }
}

/* K_c of the cell whose lower-x node is ix, lower-y node jy, between planes
 * lo (z1) and hi (z2): the eight-corner sum, G included. */
static inline void cell_from_planes(const ld *lo, const ld *hi, int nxn, int ix, int jy,
                                    ld out[NCOMP])
{
    const ld *pl[2] = {lo, hi};
    ld acc[NCOMP] = {0};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                const ld *f = pl[k] + ((size_t)(jy + j) * nxn + (ix + i)) * NCOMP;
                ld mu = corner_sign(i, j, k);
                for (int c = 0; c < NCOMP; ++c) acc[c] += mu * f[c];
            }
    for (int c = 0; c < NCOMP; ++c) out[c] = GRAV * acc[c];
}

/* ------------------------------------------------------------------------ */
/* Direct forward sum (eq. 3) at chosen stations.                            */
/* ------------------------------------------------------------------------ */

/* rho[nb][nz][ny][nx] (kg/m^3).  Stations (sp[s], sq[s]).  out[nb][nst][NCOMP].
 * Work is split over (station, chunk of consecutive layers), so each node
 * plane is evaluated once per chunk; partial sums are kept per layer and
 * reduced in layer order, so the result does not depend on the thread count
 * or the chunking. */
int orc_forward_z(int nx, int ny, int nz, double dx, double dy, double dz, const double *zedge, double h,
                  int nb, const double *rho, int nst, const int *sp, const int *sq, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || nb < 1 || nst < 0) return -1;
    if (!(dx > 0 && dy > 0 && (zedge || dz > 0) && h > 0) || check_edges(nz, zedge) != 0) return -1;
    for (int s = 0; s < nst; ++s)
        if (sp[s] < 0 || sp[s] >= nx || sq[s] < 0 || sq[s] >= ny) return -1;
    size_t nxn = (size_t)nx + 1, nyn = (size_t)ny + 1;
    size_t plane_sz = nxn * nyn * NCOMP;
    /* chunks per station: enough items to keep every thread busy */
    int nthr = orc_max_threads();
    int nchunk = (4 * nthr + nst - 1) / (nst > 0 ? nst : 1);
    if (nchunk < 1) nchunk = 1;
    if (nchunk > nz) nchunk = nz;
    int clen = (nz + nchunk - 1) / nchunk;
    nchunk = (nz + clen - 1) / clen;
    size_t nitems = (size_t)nst * nchunk;
    ld *part = (ld *)calloc((size_t)nst * nz * nb * NCOMP + 1, sizeof(ld));
    if (!part) return -2;
    int err = 0;
#pragma omp parallel
    {
        ld *lo = (ld *)malloc(plane_sz * sizeof(ld));
        ld *hi = (ld *)malloc(plane_sz * sizeof(ld));
        if (!lo || !hi) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (long it = 0; it < (long)nitems; ++it) {
            if (!lo || !hi) continue;
            int s = (int)(it / nchunk), ch = (int)(it % nchunk);
            int p = sp[s], q = sq[s];
            int n0 = ch * clen, n1 = n0 + clen < nz ? n0 + clen : nz;
            /* offsets a = l - p, l in [0,nx): x nodes (a - 1/2) dx for a in [-p, nx - p]. */
            fill_plane(lo, -p, (int)nxn, -q, (int)nyn, dx, dy, (ld)h + layer_depth(n0, dz, zedge));
            for (int n = n0; n < n1; ++n) {
                fill_plane(hi, -p, (int)nxn, -q, (int)nyn, dx, dy, (ld)h + layer_depth(n + 1, dz, zedge));
                ld *dst = part + ((size_t)s * nz + n) * nb * NCOMP;
                for (int m = 0; m < ny; ++m)
                    for (int l = 0; l < nx; ++l) {
                        ld k[NCOMP];
                        cell_from_planes(lo, hi, (int)nxn, l, m, k);
                        for (int b = 0; b < nb; ++b) {
                            ld r = rho[(((size_t)b * nz + n) * ny + m) * nx + l];
                            for (int c = 0; c < NCOMP; ++c) dst[b * NCOMP + c] += k[c] * r;
                        }
                    }
                ld *tmp = lo;
                lo = hi;
                hi = tmp;
            }
        }
        free(lo);
        free(hi);
    }
    if (err) {
        free(part);
        return err;
    }
    for (int b = 0; b < nb; ++b)
        for (int s = 0; s < nst; ++s)
            for (int c = 0; c < NCOMP; ++c) {
                ld acc = 0;
                for (int n = 0; n < nz; ++n) acc += part[(((size_t)s * nz + n) * nb + b) * NCOMP + c];
                out[((size_t)b * nst + s) * NCOMP + c] = (double)acc;
            }
    free(part);
    return 0;
}

int orc_forward(int nx, int ny, int nz, double dx, double dy, double dz, double h, int nb,
                const double *rho, int nst, const int *sp, const int *sq, double *out)
{
    return orc_forward_z(nx, ny, nz, dx, dy, dz, NULL, h, nb, rho, nst, sp, sq, out);
}

/* ------------------------------------------------------------------------ */
/* Tabulated direct sum (eq. 3 with the offset tables of eq. 7 / eq. 10).     */
/* ------------------------------------------------------------------------ */

typedef double v4d __attribute__((vector_size(32)));

/* s[j] = sum_l t[j*stride + l] r[l] for j < 3, in double: four interleaved
 * partial sums per j (l mod 4), added pairwise at the end, then the tail.
 * Three rows share each load of r; rows past nj are not read. */
static void dot_rows3(const double *t, size_t stride, int nj, const double *r, int n, double s[3])
{
    v4d a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0;
    const double *t0 = t, *t1 = nj > 1 ? t + stride : t, *t2 = nj > 2 ? t + 2 * stride : t;
    int l = 0;
    for (; l + 4 <= n; l += 4) {
        v4d x, k0, k1, k2;
        memcpy(&x, r + l, sizeof x);
        memcpy(&k0, t0 + l, sizeof k0);
        memcpy(&k1, t1 + l, sizeof k1);
        memcpy(&k2, t2 + l, sizeof k2);
        a0 += k0 * x;
        a1 += k1 * x;
        a2 += k2 * x;
    }
    s[0] = (a0[0] + a0[1]) + (a0[2] + a0[3]);
    s[1] = (a1[0] + a1[1]) + (a1[2] + a1[3]);
    s[2] = (a2[0] + a2[1]) + (a2[2] + a2[3]);
    for (; l < n; ++l) {
        s[0] += t0[l] * r[l];
        s[1] += t1[l] * r[l];
        s[2] += t2[l] * r[l];
    }
}

/* The same sum as orc_forward, d(p,q) = sum_n sum_m sum_l K_n(l-p, m-q)
 * rho(l,m,n), but each layer's kernel is first tabulated once over all
 * offsets (a, b) in [-(nx-1), nx-1] x [-(ny-1), ny-1] (translation
 * equivalence: the entry depends on the offset and the layer only), from
 * the same node-plane closed form in long double, then rounded to double.
 * The sum itself is multiply-adds only, so every station of a 256^2 x 64
 * grid, or a thousand stations of a 1024^2 x 100 grid, take seconds where
 * the per-station closed form takes hours.
 *
 * Order of the arithmetic for each station and component: the inner sum
 * over l of row m in double (dot_rows3: four interleaved partial sums), the
 * row sums added in ascending m into the layer's sum and the layers in
 * ascending n, both in long double.  The loops over rows run with the row
 * offset b = m - q outermost, so that one table row serves every station in
 * turn; for a given station that is still ascending m.  Rounding: each
 * table entry carries 2^-53 relative, each row sum at most (nx/4 + 2) 2^-53
 * of its sum of |K rho|; at nx = 1024 that bounds the result's error by
 * 3e-14 of sum |K rho| (against 1e-10 asked of the FP64 operator).
 *
 * mask: components to sum (bit c = component c); the others are returned as
 * 0.  rho[nb][nz][ny][nx], stations (sp[s], sq[s]), out[nb][nst][NCOMP].
 * Returns 0, -1 for bad arguments, -2 when memory runs out. */
int orc_forward_tab_z(int nx, int ny, int nz, double dx, double dy, double dz, const double *zedge, double h,
                      int nb, const double *rho, unsigned mask, int nst, const int *sp, const int *sq,
                      double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || nb < 1 || nst < 0) return -1;
    if (!(dx > 0 && dy > 0 && (zedge || dz > 0) && h > 0) || check_edges(nz, zedge) != 0) return -1;
    for (int s = 0; s < nst; ++s)
        if (sp[s] < 0 || sp[s] >= nx || sq[s] < 0 || sq[s] >= ny) return -1;
    int cid[NCOMP], nc = 0;
    for (int c = 0; c < NCOMP; ++c)
        if (mask & (1u << c)) cid[nc++] = c;
    if (nc == 0) return -1;
    const int na = 2 * nx - 1, nbr = 2 * ny - 1;   /* offsets a, b */
    const int nxn = 2 * nx, nyn = 2 * ny;          /* nodes (a - 1/2) dx, a in [-(nx-1), nx] */
    const size_t tsz = (size_t)na * nbr;           /* one component's table */
    ld *lo = (ld *)malloc((size_t)nxn * nyn * NCOMP * sizeof(ld));
    ld *hi = (ld *)malloc((size_t)nxn * nyn * NCOMP * sizeof(ld));
    double *tab = (double *)malloc(tsz * nc * sizeof(double));
    ld *lay = (ld *)malloc(((size_t)nst * nb * nc + 1) * sizeof(ld));
    ld *tot = (ld *)calloc((size_t)nst * nb * nc + 1, sizeof(ld));
    if (!lo || !hi || !tab || !lay || !tot) {
        free(lo); free(hi); free(tab); free(lay); free(tot);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (int jy = 0; jy < nyn; ++jy)
        fill_plane(lo + (size_t)jy * nxn * NCOMP, -(nx - 1), nxn, -(ny - 1) + jy, 1, dx, dy,
                   (ld)h + layer_depth(0, dz, zedge));
    for (int n = 0; n < nz; ++n) {
#pragma omp parallel for schedule(static)
        for (int jy = 0; jy < nyn; ++jy)
            fill_plane(hi + (size_t)jy * nxn * NCOMP, -(nx - 1), nxn, -(ny - 1) + jy, 1, dx, dy,
                       (ld)h + layer_depth(n + 1, dz, zedge));
        /* tab[j][bi][ai]: component cid[j], offset b = bi - (ny-1), a = ai - (nx-1) */
#pragma omp parallel for schedule(static)
        for (int bi = 0; bi < nbr; ++bi)
            for (int ai = 0; ai < na; ++ai) {
                ld k[NCOMP];
                cell_from_planes(lo, hi, nxn, ai, bi, k);
                for (int j = 0; j < nc; ++j) tab[j * tsz + (size_t)bi * na + ai] = (double)k[cid[j]];
            }
        for (size_t i = 0; i < (size_t)nst * nb * nc; ++i) lay[i] = 0;
        for (int b = -(ny - 1); b <= ny - 1; ++b) {
#pragma omp parallel for schedule(static)
            for (int s = 0; s < nst; ++s) {
                int m = sq[s] + b;
                if (m < 0 || m >= ny) continue;
                /* the row's entries for l = 0 .. nx-1 are the offsets a = l - p */
                const double *row = tab + (size_t)(b + ny - 1) * na + (nx - 1 - sp[s]);
                for (int bb = 0; bb < nb; ++bb) {
                    const double *rr = rho + (((size_t)bb * nz + n) * ny + m) * nx;
                    ld *dst = lay + ((size_t)s * nb + bb) * nc;
                    for (int j = 0; j < nc; j += 3) {
                        double sj[3];
                        dot_rows3(row + j * tsz, tsz, nc - j, rr, nx, sj);
                        for (int i = 0; i < 3 && j + i < nc; ++i) dst[j + i] += sj[i];
                    }
                }
            }
        }
        for (size_t i = 0; i < (size_t)nst * nb * nc; ++i) tot[i] += lay[i];
        ld *tmp = lo;
        lo = hi;
        hi = tmp;
    }
    for (int bb = 0; bb < nb; ++bb)
        for (int s = 0; s < nst; ++s) {
            double *o = out + ((size_t)bb * nst + s) * NCOMP;
            for (int c = 0; c < NCOMP; ++c) o[c] = 0;
            for (int j = 0; j < nc; ++j) o[cid[j]] = (double)tot[((size_t)s * nb + bb) * nc + j];
        }
    free(lo); free(hi); free(tab); free(lay); free(tot);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Direct adjoint sum: g(l,m,n) = sum_c sum_{p,q} G_c[(p,q),(l,m,n)] r_c(p,q) */
/* ------------------------------------------------------------------------ */

/* r[nb][NCOMP][ny][nx] indexed by component slot (unused slots may hold anything,
 * only comps in mask are read).  Cells (cl, cm, cn).  out[nb][ncell]. */
int orc_adjoint_z(int nx, int ny, int nz, double dx, double dy, double dz, const double *zedge, double h,
                  int nb, unsigned mask, const double *r, int ncell, const int *cl, const int *cm,
                  const int *cn, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || nb < 1 || ncell < 0) return -1;
    if (!(dx > 0 && dy > 0 && (zedge || dz > 0) && h > 0) || check_edges(nz, zedge) != 0) return -1;
    for (int i = 0; i < ncell; ++i)
        if (cl[i] < 0 || cl[i] >= nx || cm[i] < 0 || cm[i] >= ny || cn[i] < 0 || cn[i] >= nz)
            return -1;
    size_t nxn = (size_t)nx + 1, nyn = (size_t)ny + 1;
    size_t plane_sz = nxn * nyn * NCOMP;
    int err = 0;
#pragma omp parallel
    {
        ld *lo = (ld *)malloc(plane_sz * sizeof(ld));
        ld *hi = (ld *)malloc(plane_sz * sizeof(ld));
        if (!lo || !hi) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < ncell; ++i) {
            if (!lo || !hi) continue;
            int l = cl[i], m = cm[i], n = cn[i];
            /* a = l - p for p in [0,nx): a in [l-nx+1, l]; x nodes v in [l-nx+1, l+1]. */
            int v0 = l - nx + 1, w0 = m - ny + 1;
            fill_plane(lo, v0, (int)nxn, w0, (int)nyn, dx, dy, (ld)h + layer_depth(n, dz, zedge));
            fill_plane(hi, v0, (int)nxn, w0, (int)nyn, dx, dy, (ld)h + layer_depth(n + 1, dz, zedge));
            for (int b = 0; b < nb; ++b) {
                ld acc = 0;
                for (int q = 0; q < ny; ++q)
                    for (int p = 0; p < nx; ++p) {
                        ld k[NCOMP];
                        cell_from_planes(lo, hi, (int)nxn, (l - p) - v0, (m - q) - w0, k);
                        for (int c = 0; c < NCOMP; ++c)
                            if (mask & (1u << c))
                                acc += k[c] * r[(((size_t)b * NCOMP + c) * ny + q) * nx + p];
                    }
                out[(size_t)b * ncell + i] = (double)acc;
            }
        }
        free(lo);
        free(hi);
    }
    return err;
}

int orc_adjoint(int nx, int ny, int nz, double dx, double dy, double dz, double h, int nb,
                unsigned mask, const double *r, int ncell, const int *cl, const int *cm,
                const int *cn, double *out)
{
    return orc_adjoint_z(nx, ny, nz, dx, dy, dz, NULL, h, nb, mask, r, ncell, cl, cm, cn, out);
}

/* ------------------------------------------------------------------------ */
/* Dense kernel matrix for tiny grids (the point-element method, eq. 12).    */
/* ------------------------------------------------------------------------ */

/* out[Nd][Nm] for component comp; station i = p + q nx, cell
 * j = l + m nx + n nx ny (section 2.2's numbering, x fastest).  Every entry
 * is evaluated from the absolute positions of its own station and cell. */
int orc_dense_matrix(int nx, int ny, int nz, double dx, double dy, double dz, double h, int comp,
                     double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || comp < 0 || comp >= NCOMP) return -1;
    if (!(dx > 0 && dy > 0 && dz > 0 && h > 0)) return -1;
    long nd = (long)nx * ny, nm = (long)nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nd; ++i) {
        int p = (int)(i % nx), q = (int)(i / nx);
        ld sx = ((ld)p + (ld)0.5) * dx, sy = ((ld)q + (ld)0.5) * dy, sz = -(ld)h;
        for (long j = 0; j < nm; ++j) {
            int l = (int)(j % nx), m = (int)((j / nx) % ny), n = (int)(j / ((long)nx * ny));
            ld o[NCOMP];
            prism_ld((ld)l * dx - sx, (ld)(l + 1) * dx - sx, (ld)m * dy - sy, (ld)(m + 1) * dy - sy,
                     (ld)n * dz - sz, (ld)(n + 1) * dz - sz, o);
            out[i * nm + j] = (double)o[comp];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Uniform blocks evaluated as single merged prisms (superposition).         */
/* ------------------------------------------------------------------------ */

/* Blocks k: cells l in [blk[6k],blk[6k+1]), m in [blk[6k+2],blk[6k+3]),
 * n in [blk[6k+4],blk[6k+5]) with density val[k].  Since the closed form
 * integrates any box, a block needs one evaluation per station instead of one
 * per cell.  out[nst][NCOMP] = sum_k val[k] * K(block k). */
int orc_blocks_at_stations_z(int nx, int ny, int nz, double dx, double dy, double dz, const double *zedge,
                             double h, int nblk, const int *blk, const double *val, int nst, const int *sp,
                             const int *sq, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || nblk < 0 || nst < 0) return -1;
    if (!(dx > 0 && dy > 0 && (zedge || dz > 0) && h > 0) || check_edges(nz, zedge) != 0) return -1;
    for (int k = 0; k < nblk; ++k) {
        const int *B = blk + 6 * k;
        if (B[0] < 0 || B[1] > nx || B[0] >= B[1] || B[2] < 0 || B[3] > ny || B[2] >= B[3] ||
            B[4] < 0 || B[5] > nz || B[4] >= B[5])
            return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int s = 0; s < nst; ++s) {
        ld sx = ((ld)sp[s] + (ld)0.5) * dx, sy = ((ld)sq[s] + (ld)0.5) * dy, sz = -(ld)h;
        ld acc[NCOMP] = {0};
        for (int k = 0; k < nblk; ++k) {
            const int *B = blk + 6 * k;
            ld o[NCOMP];
            prism_ld((ld)B[0] * dx - sx, (ld)B[1] * dx - sx, (ld)B[2] * dy - sy, (ld)B[3] * dy - sy,
                     layer_depth(B[4], dz, zedge) - sz, layer_depth(B[5], dz, zedge) - sz, o);
            for (int c = 0; c < NCOMP; ++c) acc[c] += (ld)val[k] * o[c];
        }
        for (int c = 0; c < NCOMP; ++c) out[(size_t)s * NCOMP + c] = (double)acc[c];
    }
    return 0;
}

int orc_blocks_at_stations(int nx, int ny, int nz, double dx, double dy, double dz, double h,
                           int nblk, const int *blk, const double *val, int nst, const int *sp,
                           const int *sq, double *out)
{
    return orc_blocks_at_stations_z(nx, ny, nz, dx, dy, dz, NULL, h, nblk, blk, val, nst, sp, sq, out);
}
