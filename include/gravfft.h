/*
 * gravfft — fast forward operator for gravity and gravity-gradient data of a
 * 3-D prism density model observed on a horizontal plane, for MI355X (gfx950).
 *
 * The operator is the superposition of eq. 3-4 of the paper,
 *
 *     d_c(p,q) = sum_{n} sum_{l,m} K_{c,n}(l-p, m-q) rho(l,m,n),
 *
 * where K_{c,n}(a,b) is the response of the prism at offset (a,b) in layer n
 * (translation equivalence, eq. 7 and eq. 10).  Each layer block of the
 * kernel matrix is block-Toeplitz with Toeplitz blocks (section 2.2.3,
 * eq. 17-22), so it is embedded in a (Py x Px) circulant and applied in the
 * 2-D Fourier domain (eq. 18); the dense matrix is never formed.
 *
 * Geometry (section 2.1): nx*ny*nz cells of dx*dy*dz metres, z down, top of
 * the model at depth 0; one station above the centre of each surface cell at
 * height h > 0.  Components: gz and the five independent tensor components
 * gxx, gxy, gxz, gyy, gyz (eq. 1); gzz = -(gxx+gyy) is derived; and the
 * horizontal first derivatives gx, gy of the potential, whose kernel
 * matrices are BTTB as well (section 2.2.3; section 3.1 shows all nine).
 *
 * Units: density in kg/m^3; gz, gx, gy in m/s^2; tensor components in 1/s^2.  The
 * gravitational constant is 6.672e-11 N m^2/kg^2 (eq. 2).
 *
 * Layouts (x fastest, section 2.2's cell numbering):
 *     rho  [B][nz][ny][nx]          density models
 *     d    [B][C][ny][nx]           data; C = popcount(components), the
 *                                   components in ascending bit order
 *                                   ([B][nt][C][ny][nx] for a plan of nt
 *                                   observation levels, gf_plan_create_levels)
 *     r    [B][C][ny][nx]           adjoint input (same layout as d)
 *     g    [B][nz][ny][nx]          adjoint output (same layout as rho)
 * Element type: double for GF_F64, float for GF_F32.
 *
 * Ownership: a plan owns its device-resident kernel spectra (and, when
 * max_batch > 0, one internal workspace).  The caller owns every data and
 * workspace pointer; all of them are device pointers.  Data pointers must
 * be aligned to their element size and a caller's workspace to 256 bytes
 * (every hipMalloc'd or torch-allocated buffer is); otherwise the call
 * returns GF_EINVAL before anything is enqueued.  gf_forward and
 * gf_adjoint only enqueue kernels on the given HIP stream: they neither
 * allocate nor synchronise, and they return before the result is ready.
 *
 * Errors: every entry point returns a status and never aborts.  A
 * thread-local message with detail is available from gf_last_error().
 *
 * Thread safety: a plan is immutable after creation.  Calls on different
 * streams may overlap if each passes its own workspace; the internal
 * workspace (workspace == NULL) serialises the caller onto one stream.
 */
#ifndef GRAVFFT_H
#define GRAVFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_plan gf_plan;

typedef enum {
    GF_OK = 0,
    GF_EINVAL = 1,        /* bad argument (null pointer, size, geometry, mask) */
    GF_ENOMEM = 2,        /* device allocation failed (nothing leaked)          */
    GF_EDEVICE = 3,       /* HIP runtime error                                 */
    GF_EUNSUPPORTED = 4,  /* size outside the compiled transform lengths       */
    GF_EBUSY = 5          /* workspace too small for the request               */
} gf_status;

/* Component bits; output order is ascending bit order. */
enum {
    GF_GZ = 1u << 0,
    GF_GXX = 1u << 1,
    GF_GXY = 1u << 2,
    GF_GXZ = 1u << 3,
    GF_GYY = 1u << 4,
    GF_GYZ = 1u << 5,
    GF_GZZ = 1u << 6,     /* derived: -(gxx + gyy) */
    GF_GX = 1u << 7,
    GF_GY = 1u << 8,
    GF_ALL6 = 0x3Fu,
    GF_ALL7 = 0x7Fu,
    GF_ALL9 = 0x1FFu      /* gz, the six tensor components, gx, gy */
};

typedef enum {
    GF_F64 = 0,           /* FP64 spectra, transforms and accumulation          */
    GF_F32 = 1            /* FP32 spectra, transforms and accumulation; the
                             kernel table itself is always generated in FP64  */
} gf_precision;

enum { GF_OP_FORWARD = 0, GF_OP_ADJOINT = 1 };

/* Plan facts, for bindings and reports. */
typedef struct {
    int nx, ny, nz;
    int px, py;            /* circulant sizes: powers of two >= 2n-1 (eq. 10-11) */
    int n_out;             /* C: number of output components (<= 9)             */
    int n_spec;            /* number of resident spectral components (<= 8)     */
    unsigned components;   /* output mask                                       */
    unsigned spec_mask;    /* components whose spectra are resident             */
    int precision;         /* gf_precision                                      */
    int max_batch;         /* internal workspace capacity (0: none)             */
    size_t spectra_bytes;  /* resident spectra                                  */
    size_t internal_workspace_bytes;
    double plan_ms;        /* wall time of gf_plan_create (kernel table + FFTs) */
    int n_levels;          /* observation levels (1 unless gf_plan_create_levels) */
    int col_groups;        /* column-pass launches per level of a forward apply:
                              resident spectra in groups of at most six (three
                              or one where LDS holds fewer at this column
                              length), each group re-reading the row-
                              transformed density                             */
    int level_path;        /* how the levels run: 0 one plane; 1 a column pass
                              per level; 2 column passes of several levels;
                              3 the Toeplitz product in depth (the column
                              transforms once, the depth products of every
                              level per frequency, the inverse transforms once);
                              4 path 3 with the depth products through a
                              transform in depth of length 256 (FP64)        */
    int level_chunk;       /* levels per chunk of paths 3 and 4 (0 otherwise)    */
} gf_plan_info_t;

/*
 * Build a plan: generate the kernel table K_{c,n}(a,b) for every resident
 * component and layer (closed-form prism response near the station,
 * Gauss-Legendre quadrature of the point kernel beyond 8 half-diagonals,
 * all in FP64; the paper's eq. 2 family), embed it in the Py x Px circulant
 * (the three virtual grids of section 2.2.2, eq. 10-11) and keep its 2-D DFT
 * resident: one real per frequency on the quarter plane
 * kx in [0, Px/2], ky in [0, Py/2], since the spectrum of each component is
 * purely real or purely imaginary and even or odd in each frequency axis
 * (the potential-field symmetry of section 2.2).  Every output component
 * except gzz has its own spectrum; gzz reuses those of gxx and gyy.  Plans
 * with more spectra than one column-pass launch holds (six; three or one at
 * the longest FP64 transform lengths) run the column pass once per group.
 *
 *   nx, ny, nz  >= 1, nx, ny <= 2048           grid size
 *   dx, dy, dz  > 0                            cell size, metres
 *   h           > 0                            station height above the top
 *   components  nonzero subset of GF_ALL9
 *   precision   GF_F64 or GF_F32
 *   max_batch   >= 0: size of an internal workspace for up to max_batch
 *               models (0 = none; callers then pass their own workspace)
 *   hip_stream  stream for the plan-time kernels (NULL = default stream);
 *               gf_plan_create synchronises it before returning
 *   out         receives the plan (NULL on failure)
 */
gf_status gf_plan_create(int nx, int ny, int nz, double dx, double dy, double dz, double h,
                         unsigned components, int precision, int max_batch, void *hip_stream,
                         gf_plan **out);

/*
 * The same for a layered (depth-stretched) mesh: layer n spans depths
 * [z_edges[n], z_edges[n+1]] below the top instead of [n dz, (n+1) dz].  The
 * paper takes the layers uniform (section 2.1); translation equivalence
 * (eq. 7) holds within each layer whatever its thickness, so every layer
 * keeps its own BTTB block and resident spectrum and the forward and adjoint
 * calls are unchanged.
 *   z_edges  host, nz + 1 finite depths in metres, z_edges[0] >= 0 and
 *            strictly increasing (else GF_EINVAL); copied, the caller keeps
 *            ownership
 * Other arguments as gf_plan_create.
 */
gf_status gf_plan_create_layered(int nx, int ny, int nz, double dx, double dy, const double *z_edges, double h,
                                 unsigned components, int precision, int max_batch, void *hip_stream,
                                 gf_plan **out);

/*
 * The equal-dimension survey of section 2.2 (Fig. 2a): the data are
 * three-dimensional as the model is, stations on n_levels horizontal planes
 * spaced dz apart, level t (t = 0 .. n_levels-1) at height h + t dz above
 * the model top, one station above each cell centre per level.  By
 * translation equivalence in depth (eq. 10) the block of level t and layer n
 * is the single-plane block of layer n + t, so the plan holds the spectra of
 * nz + n_levels - 1 layer offsets (eq. 11's 2nz when n_levels = nz) and
 * level t sums the window of them starting at offset t.
 *   n_levels  >= 1 (1 gives the plan of gf_plan_create)
 *   d, r      [B][n_levels][C][ny][nx]; rho and g as for a single plane
 * Other arguments as gf_plan_create.  gf_debug_kernel_table and
 * gf_debug_spectrum index the nz + n_levels - 1 layer offsets; the pass
 * timing's column figure also covers all inverse row passes but the last.
 */
gf_status gf_plan_create_levels(int nx, int ny, int nz, double dx, double dy, double dz, double h, int n_levels,
                                unsigned components, int precision, int max_batch, void *hip_stream,
                                gf_plan **out);

/* Free a plan and its device memory.  NULL is accepted.  The caller must have
 * finished every call that uses the plan. */
gf_status gf_plan_destroy(gf_plan *plan);

/* Fill *info. */
gf_status gf_plan_get_info(const gf_plan *plan, gf_plan_info_t *info);

/* Resident spectra bytes (0 for NULL). */
size_t gf_plan_bytes(const gf_plan *plan);

/* Device workspace a call of op (GF_OP_FORWARD / GF_OP_ADJOINT) needs for
 * `batch` models. */
gf_status gf_workspace_bytes(const gf_plan *plan, int op, int batch, size_t *bytes);

/*
 * Forward operator d = G rho (eq. 4) for `batch` density models.
 *   rho        device, [batch][nz][ny][nx]
 *   d          device, [batch][C][ny][nx]  (written completely)
 *   workspace  device scratch of workspace_bytes >= gf_workspace_bytes(FORWARD,
 *              batch), or NULL to use the plan's internal workspace
 *              (needs batch <= max_batch)
 *   hip_stream stream to enqueue on (NULL = default stream)
 * Returns GF_EBUSY when the workspace is too small, GF_EINVAL when a pointer
 * is misaligned (see Ownership).
 */
gf_status gf_forward(gf_plan *plan, const void *rho, void *d, int batch, void *workspace,
                     size_t workspace_bytes, void *hip_stream);

/*
 * Adjoint operator g = G^T r: g(l,m,n) = sum_c sum_{p,q} K_{c,n}(l-p,m-q) r_c(p,q).
 * The inverse problem of section 2.1 (find M from G and d) iterates on it.
 *   r  device, [batch][C][ny][nx];  g  device, [batch][nz][ny][nx]
 * Other arguments as gf_forward.
 */
gf_status gf_adjoint(gf_plan *plan, const void *r, void *g, int batch, void *workspace,
                     size_t workspace_bytes, void *hip_stream);

/*
 * gf_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same operator and results as gf_forward, with the workspace taken
 * from a fixed 128 MiB array of device memory that the library reserves on
 * each device when its device code is loaded there (held until the process
 * ends).  The call itself allocates nothing.
 *   rho, d, batch, hip_stream  as gf_forward; the current device must be
 *                              the plan's device (else GF_EINVAL)
 * Returns GF_EBUSY when gf_workspace_bytes(FORWARD, batch) exceeds the
 * 128 MiB.  Every call on one device shares that device's array and the
 * workspace needs no clearing between calls; calls that overlap in time on
 * one device (other streams, other threads) race on it, so callers must
 * order them on one stream or otherwise serialise them.
 */
gf_status gf_forward_noalloc(gf_plan *plan, const void *rho, void *d, int batch, void *hip_stream);

/* Per-pass timing, for benchmarks.  When enabled, gf_forward and gf_adjoint
 * record a HIP event before and after each of their three passes (row
 * transform, column pass with the layer reduction, inverse row transform) on
 * the call's stream.  Enabling creates the events; it is not safe while a
 * call on the plan is being enqueued from another thread. */
gf_status gf_plan_set_timing(gf_plan *plan, int enable);

/* Milliseconds of the three passes of the last timed call of op
 * (GF_OP_FORWARD / GF_OP_ADJOINT): ms[0] row transform, ms[1] column pass,
 * ms[2] inverse row transform.  Waits for those events. */
gf_status gf_plan_last_pass_ms(gf_plan *plan, int op, double ms[3]);

/* Name of a status code. */
const char *gf_status_string(gf_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *gf_last_error(void);

/*
 * Test access to plan-time intermediates (synchronous; slow).
 * Kernel table of layer n as generated on the device, copied to host:
 * host_out[9][2ny-1][2nx-1] with index [c][b+ny-1][a+nx-1], component order
 * gz, gxx, gxy, gxz, gyy, gyz, gzz, gx, gy (gzz = -(gxx+gyy) from the
 * generated values); it is generated for every component whatever the
 * plan's mask.
 */
gf_status gf_debug_kernel_table(const gf_plan *plan, int n, double *host_out);

/* Resident quarter-plane spectrum of component bit `component` (one of the
 * plan's spectral components) in layer n, copied to host as double:
 * host_out[Px/2+1][Py/2+1] with index [kx][ky]; the real part for
 * gz, gxx, gxy, gyy, the imaginary part for gxz, gyz, gx, gy (unit
 * gravitational constant). */
gf_status gf_debug_spectrum(const gf_plan *plan, unsigned component, int n, double *host_out);

/*
 * Test hook: how plans of several observation levels created afterwards run
 * them.  mode 0: the path whose estimated cost is lowest (the default);
 * 1: column passes (one or several levels each); 2: the Toeplitz product in
 * depth, where the transform length allows it (column lengths >= 256);
 * 3: the same with the depth products through the transform in depth
 * (FP64 plans where also nz + levels - 1 <= 256; otherwise as 2).
 * max_chunk > 0 caps the levels per chunk of the Toeplitz path (0: its
 * default, 32 GiB of chunk buffers per model).  Process-wide.  GF_EINVAL for
 * other values.
 */
gf_status gf_debug_level_path(int mode, int max_chunk);

/*
 * Failure injection, for tests of the error paths: the nth device
 * allocation the library makes from now on (nth = 1: the next one) fails as
 * if the device were out of memory, so that the call making it returns
 * GF_ENOMEM; nth = 0 switches this off.  Process-wide, not thread-safe with
 * respect to which call meets the failure.  Returns GF_EINVAL for nth < 0.
 */
gf_status gf_debug_fail_alloc(int nth);

/* Bytes of device memory the library holds at this moment, over every plan
 * of the process (spectra, twiddles, layer edges, internal workspaces, and
 * plan-time scratch while a plan is being built). */
size_t gf_debug_live_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAVFFT_H */
