// C-ABI of the fast gravity / gravity-gradient forward operator: plan
// creation (kernel table + resident spectra), forward and adjoint calls.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gf_launch.h"
#include "gravfft.h"

namespace {

constexpr double kGrav = 6.672e-11;  // gravitational constant printed with eq. 2
constexpr int kMaxN = 2048;          // largest nx, ny (Px, Py <= 4096)

thread_local std::string g_err;

gf_status fail(gf_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

int next_pow2(long v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Gauss-Legendre nodes and weights on [-1,1] (Newton iteration on the
// Legendre polynomial from the usual cosine initial guess).
void gauss_legendre(int n, double *x, double *w)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int iter = 0; iter < 100; ++iter) {
            long double p_prev = 1, p = z;
            for (int k = 2; k <= n; ++k) {
                long double pn = ((2 * k - 1) * z * p - (k - 1) * p_prev) / k;
                p_prev = p;
                p = pn;
            }
            dp = n * (z * p - p_prev) / (z * z - 1);
            long double step = p / dp;
            z -= step;
            if (fabsl(step) < 1e-19L) break;
        }
        long double p_prev = 1, p = z;
        for (int k = 2; k <= n; ++k) {
            long double pn = ((2 * k - 1) * z * p - (k - 1) * p_prev) / k;
            p_prev = p;
            p = pn;
        }
        dp = n * (z * p - p_prev) / (z * z - 1);
        x[i] = (double)z;
        w[i] = (double)(2 / ((1 - z * z) * dp * dp));
    }
}

gf::GLRules make_rules()
{
    gf::GLRules r{};
    gauss_legendre(6, r.x, r.w);
    gauss_legendre(4, r.x + 6, r.w + 6);
    gauss_legendre(3, r.x + 10, r.w + 10);
    return r;
}

// component codes: 0 gz, 1 gxx, 2 gxy, 3 gxz, 4 gyy, 5 gyz, 6 gzz, 7 gx, 8 gy
bool is_imag(int code) { return code == 3 || code == 5 || code == 7 || code == 8; }   // odd in exactly one of x, y
bool is_yodd(int code) { return code == 2 || code == 5 || code == 8; }                // odd in y

// Every device allocation of the library goes through dev_malloc and
// dev_free, which keep the bytes held (for tests that check that failed
// calls leak nothing) and can be told to fail the n-th allocation from now
// (gf_debug_fail_alloc).
std::mutex g_alloc_mu;
std::unordered_map<void *, size_t> g_live;
size_t g_live_bytes = 0;
long g_fail_countdown = 0;

// Test hook (gf_debug_level_path): how plans created afterwards run their
// observation levels (0: by their cost estimates, 1: column passes, 2: the
// Toeplitz product, 3: the Toeplitz product through the transform in depth),
// and a cap on the Toeplitz path's levels per chunk.
std::mutex g_level_mu;
int g_level_path = 0, g_level_chunk = 0;

hipError_t dev_malloc(void **ptr, size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    *ptr = nullptr;
    if (g_fail_countdown > 0 && --g_fail_countdown == 0) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) {
        g_live[*ptr] = bytes;
        g_live_bytes += bytes;
    }
    return e;
}

void dev_free(void *ptr)
{
    if (!ptr) return;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_live.find(ptr);
    if (it != g_live.end()) {
        g_live_bytes -= it->second;
        g_live.erase(it);
    }
    (void)hipFree(ptr);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { dev_free(p); }
};

}  // namespace

struct gf_plan {
    int nx, ny, nz;
    // Observation levels: nt planes of stations at heights h + t dz,
    // t = 0..nt-1 (nt = 1: the single plane of section 2.1).  Level t sees
    // model layer n where the single-plane geometry has layer n + t, so the
    // spectra cover nzs = nz + nt - 1 layer offsets (eq. 10-11).
    int nt = 1, nzs = 0;
    double dx, dy, h;
    std::vector<double> zedge;      // nzs + 1 layer-edge depths (n dz for uniform layers)
    double *zedge_dev = nullptr;    // the same on the device, for the kernel-table kernel
    unsigned mask;
    int prec;
    int max_batch;
    int px, py, M, U, Q, QP, twlog; // M column units; U = M + 1 spectral rows of QP values
    int ldc;                        // leading dimension of column layouts (even)
    int n_out;
    int out_codes[gf::kMaxOut];
    int n_spec;
    int spec_codes[8];
    unsigned spec_mask;
    unsigned imag_mask, yodd_mask;  // over spectral slots
    // Spectral slots in groups of at most gmax (six, or three or one where
    // the transform length leaves less LDS), one column-pass launch each;
    // group g holds slots [grp_c0[g], grp_c0[g] + grp_cs[g]) and its spectra
    // are stored apart as [nzs][M+1][grp_cs[g]][QP].
    int ngrp, gmax;
    int grp_c0[8], grp_cs[8];
    gf::RowCombo out_combo;         // output o from spectral slots
    gf::RowCombo in_combo;          // adjoint: spectral slot s from input components
    void *spec = nullptr;
    size_t spec_bytes = 0;
    void *tw = nullptr;             // twiddles in the plan precision
    void *tw64 = nullptr;           // twiddles in double (plan-time transforms)
    void *iws = nullptr;
    size_t iws_bytes = 0;
    int device = 0;
    double plan_ms = 0;
    bool timing = false;
    hipEvent_t ev[2][4] = {{nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr}};
    bool ev_recorded[2] = {false, false};

    bool fp64() const { return prec == GF_F64; }
    char *spec_group(int g) const { return (char *)spec + elem() * (size_t)nzs * U * QP * grp_c0[g]; }
    // spectra of group g from spectral layer t on (the window of level t)
    char *spec_window(int g, int t) const
    {
        return spec_group(g) + elem() * (size_t)t * U * grp_cs[g] * QP;
    }
    // column passes per chunk of the adjoint (each pass of a chunk has its
    // own residual spectra and layer columns; the inverse rows sum the chunk)
    int adj_passes() const { return (nt + levels_per_pass() - 1) / levels_per_pass(); }
    int adj_chunk() const { return std::min(adj_passes(), 4); }
    // Forward of several levels per column pass (one density transform per
    // layer for all of them, spectral layers in an LDS ring): plans of up to
    // three spectra at wave-split transform lengths
    bool levels_blocked() const { return nt > 1 && n_spec <= 3 && gf::col_levels_supported(fp64(), py); }
    int levels_per_pass() const { return levels_blocked() ? std::min(nt, 6 / n_spec) : 1; }
    // slots of the forward column pass's outputs (D and Dny)
    int fwd_slots() const { return levels_per_pass() * n_spec; }
    // Observation levels as a Toeplitz product in depth (the column
    // transforms of the density or residuals once, the products of every
    // level per frequency, the inverse transforms once) where that moves
    // fewer bytes than column passes per level (or per block of levels).
    // Estimated for one model, so that the choice does not depend on the
    // batch.
    size_t spec_layer_bytes() const { return elem() * (size_t)U * n_spec * QP; }
    size_t col_slab_bytes() const { return celem() * (size_t)M * ldc; }    // one [M][ldc] slab
    size_t sp_slab_bytes() const { return celem() * (size_t)U * 2 * QP; }  // one two-row spectrum slab
    // Levels per chunk of the Toeplitz path: the chunk's output spectra and
    // columns within 32 GiB per model.
    int toep_chunk_default() const
    {
        const size_t per_level = (size_t)n_spec * (sp_slab_bytes() + col_slab_bytes());
        const size_t budget = (size_t)32 << 30;
        return (int)std::max<size_t>(1, std::min<size_t>((size_t)nt, budget / per_level));
    }
    bool toeplitz_cheaper() const
    {
        if (nt < 2 || !gf::col_spectra_supported(py)) return false;
        const double R = (double)nz * col_slab_bytes(), layer = (double)spec_layer_bytes();
        double old_bytes;
        if (levels_blocked()) {
            const int per = levels_per_pass();
            old_bytes = (double)((nt + per - 1) / per) * (R + (nz + per - 1) * layer);
        } else {
            old_bytes = (double)nt * (ngrp * R + nz * layer);
        }
        const int tc = toep_chunk_default(), nch = (nt + tc - 1) / tc;
        const double X = (double)nz * sp_slab_bytes();
        const double new_bytes = X + nch * (ngrp * X + (nz + tc - 1) * layer) + 2.0 * nt * n_spec * sp_slab_bytes();
        return new_bytes < old_bytes;
    }
    bool toep = false;              // decided at creation
    int toep_tc = 1;
    // the Toeplitz path's depth products through the transform in depth
    // (decided at creation), with its plan-time values Kz, per group
    // [U][Cs][tile][129][8] complex (positions in tiles of 8), groups one after the other
    bool zdepth = false;
    void *kz = nullptr;
    size_t kz_bytes = 0;
    char *kz_group(int g) const { return (char *)kz + 2 * elem() * gf::levelz_values(U, grp_c0[g], QP); }
    // Depth products of one component over all (row, half, position)
    // sequences of the 1024^2 x 100, 100-level survey in FP64, measured: the
    // direct Toeplitz product 3.8 ms (it scales with nz * nt), the transform
    // in depth 4.0 ms for the inputs' transform and staging plus 1.6 ms per
    // component (independent of nz and nt up to nz + nt - 1 = 256).  FP32
    // keeps the direct product: the transform in depth rounds relative to the
    // whole depth sequence, which leaves levels far above the model with
    // about 1e-5 of their own size in FP32 (1e-11 in FP64).
    bool depth_transform_cheaper() const
    {
        const double direct = 3.8e-4 * n_spec * nz * nt;
        const double zt = 4.0 + 1.6 * n_spec;
        return zt < direct;
    }
    bool levels_toeplitz() const { return toep; }
    int toep_chunk() const { return toep_tc; }
    unsigned grp_bits(unsigned m, int g) const { return (m >> grp_c0[g]) & ((1u << grp_cs[g]) - 1u); }
    size_t elem() const { return fp64() ? sizeof(double) : sizeof(float); }
    size_t celem() const { return 2 * elem(); }
    int slot_of(int code) const
    {
        for (int s = 0; s < n_spec; ++s)
            if (spec_codes[s] == code) return s;
        return -1;
    }
    int out_of(int code) const
    {
        for (int o = 0; o < n_out; ++o)
            if (out_codes[o] == code) return o;
        return -1;
    }
    // Layer split of the forward column pass, and layers per split.  Chosen
    // for one model and used for every batch size, so that a model's result
    // does not depend on the batch it is computed in.
    // Units of the main column grid: the px/2 main units when the Nyquist
    // unit runs apart (in layer chunks), else all px/2 + 1.
    long main_units() const { return gf::col_nyquist_apart(py) ? (long)M : (long)U; }
    // Layer chunks of the Nyquist unit when it runs apart: up to 32 chunks.
    void nyq_split(int *Sny, int *lps_ny) const
    {
        if (!gf::col_nyquist_apart(py)) {
            *Sny = 0;
            *lps_ny = 0;
            return;
        }
        const int target = std::min(nz, 32);
        const int l = (nz + target - 1) / target;
        *lps_ny = l;
        *Sny = (nz + l - 1) / l;
    }
    size_t nyq_bytes(int B) const
    {
        int Sny, l;
        nyq_split(&Sny, &l);
        return elem() * (size_t)Sny * B * fwd_slots() * ldc;
    }
    void fwd_split(int /*B*/, int *S, int *lps) const
    {
        const int G = gf::col_forward_groups(fp64(), py);
        const long nblk = (main_units() + G - 1) / G;
        const int cap = gf::col_forward_capacity(fp64(), py, grp_cs[0], 1);
        // cost in units of one layer of one round of resident workgroups;
        // each split adds a partial-sum write and read (~beta layers)
        const double per_layer = (double)n_spec * Q + 2.0 * ny;
        const double beta = 4.0 * n_spec * ny / per_layer;
        int best = 1;
        double best_cost = 1e300;
        for (int s = 1; s <= nz && s <= 32; ++s) {
            const long l = (nz + s - 1) / s;
            if ((long)(s - 1) * l >= nz) continue;  // empty split
            const double rounds = std::ceil((double)nblk * s / cap);
            const double cost = rounds * l + beta * s * (double)nblk / cap;
            if (cost < best_cost * 0.999) {
                best_cost = cost;
                best = s;
            }
        }
        *S = best;
        *lps = (nz + best - 1) / best;
    }
    void adj_split(int B, int *S, int *lps) const
    {
        const int G = gf::col_forward_groups(fp64(), py);
        const long nblk = (main_units() * B + G - 1) / G;
        const int cap = gf::col_forward_capacity(fp64(), py, grp_cs[0], B);
        long s = (2L * cap + nblk - 1) / nblk;
        if (s < 1) s = 1;
        if (s > nz) s = nz;
        long l = (nz + s - 1) / s;
        s = (nz + l - 1) / l;
        *S = (int)s;
        *lps = (int)l;
    }
    size_t ws_bytes(int op, int B) const
    {
        if (levels_toeplitz()) {
            // forward: R [B][nz] cols, X [B][nz] spectra, Dh [B][tc][n_spec] spectra, D [B][tc][n_spec] cols;
            // adjoint: R [B][tc][n_spec] cols, X [B][tc][n_spec] spectra, Gh [B][nz] spectra, Gt [B][nz] cols
            const size_t tc = (size_t)toep_chunk();
            return (size_t)B * (nz + tc * n_spec) * (col_slab_bytes() + sp_slab_bytes());
        }
        if (op == GF_OP_FORWARD) {
            int S, l;
            fwd_split(B, &S, &l);
            return celem() * (size_t)M * ldc * ((size_t)B * nz + (size_t)S * B * fwd_slots()) + nyq_bytes(B);
        }
        return celem() * (size_t)M * ldc * (size_t)adj_chunk() * ((size_t)B * fwd_slots() + (size_t)ngrp * B * nz);
    }
};

namespace {

gf_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GF_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(GF_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(GF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
std::vector<T> twiddle_table(int n)
{
    std::vector<T> v(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < n; ++m) {
        const long double a = -2 * pi * (long double)m / (long double)n;
        v[2 * (size_t)m] = (T)cosl(a);
        v[2 * (size_t)m + 1] = (T)sinl(a);
    }
    return v;
}

gf::KgenGeom kgen_geom(const gf_plan *p)
{
    gf::KgenGeom g{};
    g.nx = p->nx;
    g.ny = p->ny;
    g.px = p->px;
    g.py = p->py;
    g.dx = p->dx;
    g.dy = p->dy;
    g.zedge = p->zedge_dev;
    g.h = p->h;
    g.t_analytic = 8.0;
    g.t_gl6 = 24.0;
    g.t_gl4 = 80.0;
    return g;
}

gf_status build_spectra(gf_plan *p, hipStream_t st)
{
    const size_t field = (size_t)p->py * p->px;
    const size_t per_pair = field * sizeof(double) + (size_t)p->M * p->py * 2 * sizeof(double);
    const size_t budget = (size_t)2 << 30;
    int nl = (int)(budget / (per_pair * p->grp_cs[0]));
    if (nl < 1) nl = 1;
    if (nl > p->nzs) nl = p->nzs;
    DevBuf E, Rk;
    gf_status s;
    if ((s = hip_check(dev_malloc((void **)&E.p, field * sizeof(double) * nl * p->grp_cs[0]), "kernel field")) != GF_OK)
        return s;
    if ((s = hip_check(dev_malloc((void **)&Rk.p, (size_t)p->M * p->py * 2 * sizeof(double) * nl * p->grp_cs[0]),
                       "kernel row spectra")) != GF_OK)
        return s;
    const gf::KgenGeom g = kgen_geom(p);
    const gf::GLRules gl = make_rules();
    gf::RowCombo ident{};
    ident.identity = 1;
    for (int gr = 0; gr < p->ngrp; ++gr) {
        const int cs = p->grp_cs[gr];
        for (int n0 = 0; n0 < p->nzs; n0 += nl) {
            const int nlc = std::min(nl, p->nzs - n0);
            const int npair = nlc * cs;
            if ((s = hip_check(hipMemsetAsync(E.p, 0, field * sizeof(double) * npair, st), "memset")) != GF_OK)
                return s;
            if (gf::launch_kgen_field(E.p, nlc, n0, cs, p->spec_codes + p->grp_c0[gr], g, gl, st) != 0)
                return fail(GF_EDEVICE, "kernel table launch failed");
            if (gf::launch_row_r2c(true, p->px, E.p, p->px, p->px, p->py, p->py, npair, npair, 1, ident, Rk.p,
                                   p->tw64, p->twlog, st) != 0)
                return fail(GF_EDEVICE, "kernel row transform launch failed");
            if (gf::launch_col_kgen(p->fp64(), p->py, Rk.p, p->spec_group(gr), nlc, n0, cs, p->nzs, p->M,
                                    p->grp_bits(p->imag_mask, gr), p->grp_bits(p->yodd_mask, gr), p->tw64,
                                    p->twlog, st) != 0)
                return fail(GF_EDEVICE, "kernel column transform launch failed");
        }
    }
    return hip_check(hipStreamSynchronize(st), "plan synchronise");
}

void mark(gf_plan *p, int op, int i, hipStream_t st)
{
    if (!p->timing) return;
    (void)hipEventRecord(p->ev[op][i], st);
    if (i == 3) p->ev_recorded[op] = true;
}

void free_plan(gf_plan *p)
{
    if (!p) return;
    for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 4; ++i)
            if (p->ev[o][i]) (void)hipEventDestroy(p->ev[o][i]);
    dev_free(p->spec);
    dev_free(p->kz);
    dev_free(p->tw);
    if (p->tw64 != p->tw) dev_free(p->tw64);
    dev_free(p->iws);
    dev_free(p->zedge_dev);
    delete p;
}

}  // namespace

// Workspace of gf_forward_noalloc: a fixed array in device memory, one per
// device, reserved when the library's device code is loaded on it and held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it names a stand-in, not the device address); it uses
// the device address looked up once per device below.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on each device).
gf_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(GF_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GF_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return GF_OK;
}

}  // namespace

extern "C" {

const char *gf_status_string(gf_status s)
{
    switch (s) {
    case GF_OK: return "GF_OK";
    case GF_EINVAL: return "GF_EINVAL";
    case GF_ENOMEM: return "GF_ENOMEM";
    case GF_EDEVICE: return "GF_EDEVICE";
    case GF_EUNSUPPORTED: return "GF_EUNSUPPORTED";
    case GF_EBUSY: return "GF_EBUSY";
    }
    return "GF_UNKNOWN";
}

const char *gf_last_error(void) { return g_err.c_str(); }

gf_status gf_debug_level_path(int mode, int max_chunk)
{
    if (mode < 0 || mode > 3 || max_chunk < 0) return fail(GF_EINVAL, "bad level path %d / chunk %d", mode, max_chunk);
    std::lock_guard<std::mutex> lk(g_level_mu);
    g_level_path = mode;
    g_level_chunk = max_chunk;
    return GF_OK;
}

gf_status gf_debug_fail_alloc(int nth)
{
    if (nth < 0) return fail(GF_EINVAL, "nth must be >= 0");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_fail_countdown = nth;
    return GF_OK;
}

size_t gf_debug_live_bytes(void)
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_live_bytes;
}

// Shared by the constructors: nt observation levels; `edges` holds the
// nz + nt layer-edge depths of the nz + nt - 1 spectral layers, already
// checked.
static gf_status create_plan(int nx, int ny, int nz, int nt, double dx, double dy, const double *edges, double h,
                             unsigned components, int precision, int max_batch, void *hip_stream,
                             gf_plan **out)
{
    if (!(dx > 0) || !(dy > 0) || !std::isfinite(dx) || !std::isfinite(dy))
        return fail(GF_EINVAL, "cell sizes must be positive and finite");
    if (!(h > 0) || !std::isfinite(h)) return fail(GF_EINVAL, "station height h must be > 0");
    if (components == 0 || (components & ~(unsigned)GF_ALL9))
        return fail(GF_EINVAL, "bad component mask 0x%x", components);
    if (precision != GF_F64 && precision != GF_F32) return fail(GF_EINVAL, "bad precision %d", precision);
    if (max_batch < 0) return fail(GF_EINVAL, "max_batch must be >= 0");
    if ((long)nz * nx * ny > (1L << 31)) return fail(GF_EUNSUPPORTED, "model too large");

    hipStream_t st = (hipStream_t)hip_stream;
    const auto t0 = std::chrono::steady_clock::now();
    gf_plan *p = new (std::nothrow) gf_plan();
    if (!p) return fail(GF_ENOMEM, "host allocation");
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->nt = nt;
    p->nzs = nz + nt - 1;
    p->dx = dx;
    p->dy = dy;
    p->zedge.assign(edges, edges + p->nzs + 1);
    p->h = h;
    p->mask = components;
    p->prec = precision;
    p->max_batch = max_batch;
    // circulant sizes: any P >= 2n-1 embeds the Toeplitz levels exactly
    p->px = std::max(16, next_pow2(2L * nx - 1));
    p->py = std::max(16, next_pow2(2L * ny - 1));
    p->M = p->px / 2;
    p->U = p->M + 1;
    p->Q = p->py / 2 + 1;
    p->QP = gf::spec_row_pitch(precision == GF_F64, p->py);
    p->ldc = ny + (ny & 1);
    p->twlog = log2i(std::max(p->px, p->py));
    (void)hipGetDevice(&p->device);

    p->n_out = 0;
    for (int c = 0; c < gf::kMaxOut; ++c)
        if (components & (1u << c)) p->out_codes[p->n_out++] = c;
    p->spec_mask = components & ~(unsigned)GF_GZZ;
    if (components & GF_GZZ) p->spec_mask |= GF_GXX | GF_GYY;
    p->n_spec = 0;
    p->imag_mask = p->yodd_mask = 0;
    for (int c = 0; c < gf::kMaxOut; ++c)
        if (p->spec_mask & (1u << c)) {
            const int s = p->n_spec++;
            p->spec_codes[s] = c;
            if (is_imag(c)) p->imag_mask |= 1u << s;
            if (is_yodd(c)) p->yodd_mask |= 1u << s;
        }
    p->gmax = 0;
    for (int c : {gf::kColMaxSpec, 3, 1})
        if (gf::col_supported(precision == GF_F64, p->py, c)) {
            p->gmax = c;
            break;
        }
    if (p->gmax == 0) {
        free_plan(p);
        return fail(GF_EUNSUPPORTED, "transform length %d does not fit in LDS", p->py);
    }
    p->ngrp = (p->n_spec + p->gmax - 1) / p->gmax;
    for (int g = 0; g < p->ngrp; ++g) {
        p->grp_c0[g] = g * p->gmax;
        p->grp_cs[g] = std::min(p->gmax, p->n_spec - p->grp_c0[g]);
    }
    {
        std::lock_guard<std::mutex> lk(g_level_mu);
        if (nt > 1 && gf::col_spectra_supported(p->py))
            p->toep = g_level_path == 2 || g_level_path == 3 || (g_level_path == 0 && p->toeplitz_cheaper());
        p->zdepth = p->toep && p->fp64() && gf::levelz_supported(p->nzs) && p->twlog >= 8 &&
                    (g_level_path == 3 || (g_level_path == 0 && p->depth_transform_cheaper()));
        p->toep_tc = p->toep_chunk_default();
        if (g_level_chunk > 0) p->toep_tc = std::min(p->toep_tc, g_level_chunk);
    }
    std::memset(&p->out_combo, 0, sizeof(p->out_combo));
    for (int o = 0; o < p->n_out; ++o) {
        const int code = p->out_codes[o];
        if (code != 6) {
            p->out_combo.nterm[o] = 1;
            p->out_combo.src[o][0] = p->slot_of(code);
            p->out_combo.w[o][0] = 1.0;
        } else {
            p->out_combo.nterm[o] = 2;
            p->out_combo.src[o][0] = p->slot_of(1);
            p->out_combo.src[o][1] = p->slot_of(4);
            p->out_combo.w[o][0] = -1.0;
            p->out_combo.w[o][1] = -1.0;
        }
    }
    std::memset(&p->in_combo, 0, sizeof(p->in_combo));
    for (int s = 0; s < p->n_spec; ++s) {
        const int code = p->spec_codes[s];
        int k = 0;
        const int o = p->out_of(code);
        if (o >= 0) {
            p->in_combo.src[s][k] = o;
            p->in_combo.w[s][k] = 1.0;
            ++k;
        }
        const int oz = p->out_of(6);
        if ((code == 1 || code == 4) && oz >= 0) {
            p->in_combo.src[s][k] = oz;
            p->in_combo.w[s][k] = -1.0;
            ++k;
        }
        p->in_combo.nterm[s] = k;
    }

    gf_status s;
    if ((s = hip_check(dev_malloc((void **)&p->zedge_dev, (p->nzs + 1) * sizeof(double)), "layer edges")) != GF_OK ||
        (s = hip_check(hipMemcpy(p->zedge_dev, p->zedge.data(), (p->nzs + 1) * sizeof(double), hipMemcpyHostToDevice),
                       "layer edges")) != GF_OK) {
        free_plan(p);
        return s;
    }
    const int tl = 1 << p->twlog;
    {
        auto t64 = twiddle_table<double>(tl);
        if ((s = hip_check(dev_malloc((void **)&p->tw64, t64.size() * sizeof(double)), "twiddles")) != GF_OK) {
            free_plan(p);
            return s;
        }
        if ((s = hip_check(hipMemcpy(p->tw64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice),
                           "twiddles")) != GF_OK) {
            free_plan(p);
            return s;
        }
        if (p->fp64()) {
            p->tw = p->tw64;
        } else {
            auto t32 = twiddle_table<float>(tl);
            if ((s = hip_check(dev_malloc((void **)&p->tw, t32.size() * sizeof(float)), "twiddles")) != GF_OK ||
                (s = hip_check(hipMemcpy(p->tw, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice),
                               "twiddles")) != GF_OK) {
                free_plan(p);
                return s;
            }
        }
    }
    for (int g = 0; g < p->ngrp; ++g)
        if (!gf::col_supported(p->fp64(), p->py, p->grp_cs[g])) {
            free_plan(p);
            return fail(GF_EUNSUPPORTED, "transform length %d with %d components does not fit in LDS", p->py,
                        p->grp_cs[g]);
        }
    p->spec_bytes = (size_t)p->nzs * p->U * p->n_spec * p->QP * p->elem();
    if ((s = hip_check(dev_malloc((void **)&p->spec, p->spec_bytes), "spectra")) != GF_OK) {
        free_plan(p);
        return s;
    }
    if ((s = build_spectra(p, st)) != GF_OK) {
        free_plan(p);
        return s;
    }
    if (p->zdepth) {
        p->kz_bytes = 2 * p->elem() * gf::levelz_values(p->U, p->n_spec, p->QP);
        if ((s = hip_check(dev_malloc((void **)&p->kz, p->kz_bytes), "depth-transformed spectra")) != GF_OK) {
            free_plan(p);
            return s;
        }
        // zero first: the last position tile of each row has padding slots
        if ((s = hip_check(hipMemsetAsync(p->kz, 0, p->kz_bytes, st), "memset")) != GF_OK) {
            free_plan(p);
            return s;
        }
        for (int gr = 0; gr < p->ngrp; ++gr)
            if (gf::launch_levelz_kgen(p->spec_group(gr), p->kz_group(gr), p->nzs, p->U, p->grp_cs[gr],
                                       p->QP, p->tw64, p->twlog, st) != 0) {
                free_plan(p);
                return fail(GF_EDEVICE, "depth transform launch failed");
            }
        if ((s = hip_check(hipStreamSynchronize(st), "plan synchronise")) != GF_OK) {
            free_plan(p);
            return s;
        }
    }
    if (max_batch > 0) {
        p->iws_bytes = std::max(p->ws_bytes(GF_OP_FORWARD, max_batch), p->ws_bytes(GF_OP_ADJOINT, max_batch));
        if ((s = hip_check(dev_malloc((void **)&p->iws, p->iws_bytes), "internal workspace")) != GF_OK) {
            free_plan(p);
            return s;
        }
    }
    p->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return GF_OK;
}

static gf_status check_grid(int nx, int ny, int nz, gf_plan **out)
{
    g_err.clear();
    if (!out) return fail(GF_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(GF_EINVAL, "grid sizes must be >= 1 (got %d,%d,%d)", nx, ny, nz);
    if (nx > kMaxN || ny > kMaxN)
        return fail(GF_EUNSUPPORTED, "nx, ny must be <= %d (got %d,%d)", kMaxN, nx, ny);
    if ((long)nz * nx * ny > (1L << 31)) return fail(GF_EUNSUPPORTED, "model too large");
    return GF_OK;
}

gf_status gf_plan_create(int nx, int ny, int nz, double dx, double dy, double dz, double h,
                         unsigned components, int precision, int max_batch, void *hip_stream,
                         gf_plan **out)
{
    gf_status s = check_grid(nx, ny, nz, out);
    if (s != GF_OK) return s;
    if (!(dz > 0) || !std::isfinite(dz)) return fail(GF_EINVAL, "cell sizes must be positive and finite");
    std::vector<double> edges(nz + 1);
    for (int n = 0; n <= nz; ++n) edges[n] = n * dz;
    return create_plan(nx, ny, nz, 1, dx, dy, edges.data(), h, components, precision, max_batch, hip_stream, out);
}

gf_status gf_plan_create_levels(int nx, int ny, int nz, double dx, double dy, double dz, double h, int n_levels,
                                unsigned components, int precision, int max_batch, void *hip_stream,
                                gf_plan **out)
{
    gf_status s = check_grid(nx, ny, nz, out);
    if (s != GF_OK) return s;
    if (!(dz > 0) || !std::isfinite(dz)) return fail(GF_EINVAL, "cell sizes must be positive and finite");
    if (n_levels < 1) return fail(GF_EINVAL, "n_levels must be >= 1 (got %d)", n_levels);
    if (((long)nz + n_levels - 1) * nx * ny > (1L << 31)) return fail(GF_EUNSUPPORTED, "model too large");
    const int nzs = nz + n_levels - 1;
    std::vector<double> edges(nzs + 1);
    for (int n = 0; n <= nzs; ++n) edges[n] = n * dz;
    return create_plan(nx, ny, nz, n_levels, dx, dy, edges.data(), h, components, precision, max_batch, hip_stream,
                       out);
}

gf_status gf_plan_create_layered(int nx, int ny, int nz, double dx, double dy, const double *z_edges, double h,
                                 unsigned components, int precision, int max_batch, void *hip_stream,
                                 gf_plan **out)
{
    gf_status s = check_grid(nx, ny, nz, out);
    if (s != GF_OK) return s;
    if (!z_edges) return fail(GF_EINVAL, "z_edges is NULL");
    if (!(z_edges[0] >= 0) || !std::isfinite(z_edges[0])) return fail(GF_EINVAL, "z_edges[0] must be >= 0");
    for (int n = 0; n < nz; ++n)
        if (!(z_edges[n + 1] > z_edges[n]) || !std::isfinite(z_edges[n + 1]))
            return fail(GF_EINVAL, "z_edges must increase strictly (at %d)", n + 1);
    return create_plan(nx, ny, nz, 1, dx, dy, z_edges, h, components, precision, max_batch, hip_stream, out);
}

gf_status gf_plan_destroy(gf_plan *plan)
{
    free_plan(plan);
    return GF_OK;
}

gf_status gf_plan_get_info(const gf_plan *p, gf_plan_info_t *info)
{
    if (!p || !info) return fail(GF_EINVAL, "NULL argument");
    info->nx = p->nx;
    info->ny = p->ny;
    info->nz = p->nz;
    info->n_levels = p->nt;
    info->col_groups = p->ngrp;
    info->px = p->px;
    info->py = p->py;
    info->n_out = p->n_out;
    info->n_spec = p->n_spec;
    info->components = p->mask;
    info->spec_mask = p->spec_mask;
    info->precision = p->prec;
    info->max_batch = p->max_batch;
    info->spectra_bytes = p->spec_bytes + p->kz_bytes;
    info->internal_workspace_bytes = p->iws_bytes;
    info->plan_ms = p->plan_ms;
    info->level_path = p->nt < 2 ? 0 : (p->toep ? (p->zdepth ? 4 : 3) : (p->levels_blocked() ? 2 : 1));
    info->level_chunk = p->toep ? p->toep_tc : 0;
    return GF_OK;
}

size_t gf_plan_bytes(const gf_plan *p) { return p ? p->spec_bytes + p->kz_bytes : 0; }

gf_status gf_workspace_bytes(const gf_plan *p, int op, int batch, size_t *bytes)
{
    if (!p || !bytes) return fail(GF_EINVAL, "NULL argument");
    if (op != GF_OP_FORWARD && op != GF_OP_ADJOINT) return fail(GF_EINVAL, "bad op %d", op);
    if (batch < 1) return fail(GF_EINVAL, "batch must be >= 1");
    *bytes = p->ws_bytes(op, batch);
    return GF_OK;
}

// Data pointers must be aligned to their element (the kernels take vector
// accesses only where the pointer allows them); a caller's workspace to 256
// bytes, as every device allocation is (its slabs are read and written as
// 16-byte vectors).
static gf_status check_align(const gf_plan *p, const void *in, const void *out)
{
    const uintptr_t e = (uintptr_t)p->elem();
    if (((uintptr_t)in | (uintptr_t)out) & (e - 1))
        return fail(GF_EINVAL, "data pointers must be aligned to their %u-byte element", (unsigned)e);
    return GF_OK;
}

static gf_status pick_ws(gf_plan *p, int op, int batch, void *&ws, size_t ws_bytes)
{
    const size_t need = p->ws_bytes(op, batch);
    if (ws && ((uintptr_t)ws & 255u))
        return fail(GF_EINVAL, "workspace must be 256-byte aligned");
    if (!ws) {
        if (!p->iws || batch > p->max_batch)
            return fail(GF_EBUSY, "no workspace given and batch %d exceeds the internal workspace (max_batch %d)",
                        batch, p->max_batch);
        ws = p->iws;
        return GF_OK;
    }
    if (ws_bytes < need)
        return fail(GF_EBUSY, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, need);
    return GF_OK;
}

gf_status gf_forward(gf_plan *p, const void *rho, void *d, int batch, void *workspace,
                     size_t workspace_bytes, void *hip_stream)
{
    if (!p || !rho || !d) return fail(GF_EINVAL, "NULL argument");
    if (batch < 1) return fail(GF_EINVAL, "batch must be >= 1");
    gf_status s = check_align(p, rho, d);
    if (s != GF_OK) return s;
    s = pick_ws(p, GF_OP_FORWARD, batch, workspace, workspace_bytes);
    if (s != GF_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    int S, lps;
    p->fwd_split(batch, &S, &lps);
    char *R = (char *)workspace;
    char *D = R + p->celem() * (size_t)batch * p->nz * p->M * p->ldc;
    gf::NyqSplit nq{nullptr, 0, 0};
    p->nyq_split(&nq.Sny, &nq.lps_ny);
    if (nq.Sny > 0) nq.Dny = D + p->celem() * (size_t)S * batch * p->fwd_slots() * p->M * p->ldc;
    gf::RowCombo ident{};
    ident.identity = 1;
    mark(p, GF_OP_FORWARD, 0, st);
    if (gf::launch_row_r2c(p->fp64(), p->px, rho, p->nx, p->nx, p->ny, p->ldc, p->nz, p->nz, batch, ident, R,
                           p->tw, p->twlog, st) != 0)
        return fail(GF_EDEVICE, "row transform launch: %s", hipGetErrorString(hipGetLastError()));
    mark(p, GF_OP_FORWARD, 1, st);
    // level t: the layer sum over the spectra window starting at spectral
    // layer t, into d[b][t]
    const size_t plane = (size_t)p->nx * p->ny;
    const long dstride = (long)p->nt * p->n_out * (long)plane;
    const double scale = kGrav / ((double)p->py * p->M);
    if (p->levels_toeplitz()) {
        // the density spectra once; per chunk of levels the depth products of
        // every group, the inverse column transforms and the inverse rows of
        // each level
        const int tcm = p->toep_chunk();
        char *X = R + p->col_slab_bytes() * (size_t)batch * p->nz;
        char *Dh = X + p->sp_slab_bytes() * (size_t)batch * p->nz;
        char *Dc = Dh + p->sp_slab_bytes() * (size_t)batch * tcm * p->n_spec;
        if (gf::launch_col_spectra(p->fp64(), p->py, R, X, batch, p->nz, p->M, p->ny, p->ldc, p->tw, p->twlog, st) != 0)
            return fail(GF_EDEVICE, "column spectra launch: %s", hipGetErrorString(hipGetLastError()));
        const gf::NyqSplit none{nullptr, 0, 0};
        for (int t0 = 0; t0 < p->nt; t0 += tcm) {
            const int tc = std::min(tcm, p->nt - t0);
            for (int gr = 0; gr < p->ngrp; ++gr) {
                char *Dg = Dh + p->sp_slab_bytes() * (size_t)p->grp_c0[gr];
                const int e = p->zdepth
                                  ? gf::launch_levelz_forward(X, p->kz_group(gr), Dg, batch, p->nz, t0, tc,
                                                              p->nt, p->U, p->QP, p->grp_cs[gr], p->n_spec,
                                                              p->grp_bits(p->imag_mask, gr),
                                                              p->grp_bits(p->yodd_mask, gr), p->tw, p->twlog, st)
                                  : gf::launch_levels_forward(p->fp64(), p->py, X, p->spec_window(gr, t0), Dg, batch,
                                                              p->nz, tc, p->M, p->grp_cs[gr], p->n_spec,
                                                              p->grp_bits(p->imag_mask, gr),
                                                              p->grp_bits(p->yodd_mask, gr), st);
                if (e != 0) return fail(GF_EDEVICE, "depth product launch: %s", hipGetErrorString(hipGetLastError()));
            }
            const int slots = tc * p->n_spec;
            if (gf::launch_col_inverse(p->fp64(), p->py, Dh, Dc, batch, slots, p->M, p->ny, p->ldc, p->tw, p->twlog,
                                       st) != 0)
                return fail(GF_EDEVICE, "inverse column launch: %s", hipGetErrorString(hipGetLastError()));
            if (t0 + tc == p->nt) mark(p, GF_OP_FORWARD, 2, st);
            // the inverse rows of every level of the chunk in one launch per
            // model (levels are consecutive items of n_spec slabs in Dc and of
            // n_out planes in d); one launch for all models when the chunk is
            // every level
            const int nitems = tc == p->nt ? batch * tc : tc;
            for (int b0 = 0; b0 < batch; b0 += nitems / tc) {
                if (gf::launch_row_c2r(p->fp64(), p->px, Dc + p->col_slab_bytes() * (size_t)b0 * slots,
                                       (long)nitems * p->n_spec * p->M * p->ldc, 1, p->n_spec, p->ny, p->ldc, p->n_out,
                                       nitems, p->out_combo, none,
                                       (char *)d + p->elem() * ((size_t)b0 * p->nt + t0) * p->n_out * plane, p->nx,
                                       scale, p->tw, p->twlog, st, (long)p->n_out * plane, false) != 0)
                    return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
            }
        }
        mark(p, GF_OP_FORWARD, 3, st);
        return GF_OK;
    }
    if (p->levels_blocked()) {
        // passes of up to levels_per_pass() levels; level j of a pass is
        // slots [j Cs, (j+1) Cs) of its D and Dny
        const int per = p->levels_per_pass();
        for (int t0 = 0; t0 < p->nt; t0 += per) {
            const int nlev = std::min(per, p->nt - t0);
            const int slots = nlev * p->n_spec;
            if (gf::launch_col_forward_levels(p->fp64(), p->py, R, p->spec_window(0, t0), D, batch, p->nz, p->M, p->ny,
                                              p->ldc, p->n_spec, nlev, S, lps, nq, p->imag_mask, p->yodd_mask, p->tw,
                                              p->twlog, st) != 0)
                return fail(GF_EDEVICE, "column pass launch: %s", hipGetErrorString(hipGetLastError()));
            if (t0 + nlev == p->nt) mark(p, GF_OP_FORWARD, 2, st);
            for (int j = 0; j < nlev; ++j) {
                gf::RowCombo cmb = p->out_combo;
                for (int o = 0; o < p->n_out; ++o)
                    for (int i = 0; i < cmb.nterm[o]; ++i) cmb.src[o][i] += j * p->n_spec;
                if (gf::launch_row_c2r(p->fp64(), p->px, D, (long)batch * slots * p->M * p->ldc, S, slots, p->ny,
                                       p->ldc, p->n_out, batch, cmb, nq,
                                       (char *)d + p->elem() * (size_t)(t0 + j) * p->n_out * plane, p->nx, scale,
                                       p->tw, p->twlog, st, dstride, false) != 0)
                    return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
            }
        }
        mark(p, GF_OP_FORWARD, 3, st);
        return GF_OK;
    }
    for (int t = 0; t < p->nt; ++t) {
        for (int gr = 0; gr < p->ngrp; ++gr) {
            const int c0 = p->grp_c0[gr];
            gf::NyqSplit nqg = nq;
            if (nqg.Dny) nqg.Dny = (char *)nqg.Dny + p->elem() * (size_t)c0 * p->ldc;
            if (gf::launch_col_forward(p->fp64(), p->py, R, p->spec_window(gr, t),
                                       D + p->celem() * (size_t)c0 * p->M * p->ldc, batch, p->nz, p->M, p->ny, p->ldc,
                                       p->grp_cs[gr], p->n_spec, S, lps, nqg, p->grp_bits(p->imag_mask, gr),
                                       p->grp_bits(p->yodd_mask, gr), p->tw, p->twlog, st) != 0)
                return fail(GF_EDEVICE, "column pass launch: %s", hipGetErrorString(hipGetLastError()));
        }
        if (t == p->nt - 1) mark(p, GF_OP_FORWARD, 2, st);
        if (gf::launch_row_c2r(p->fp64(), p->px, D, (long)batch * p->n_spec * p->M * p->ldc, S, p->n_spec, p->ny,
                               p->ldc, p->n_out, batch, p->out_combo, nq,
                               (char *)d + p->elem() * (size_t)t * p->n_out * plane, p->nx, scale, p->tw, p->twlog,
                               st, dstride, false) != 0)
            return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
    }
    mark(p, GF_OP_FORWARD, 3, st);
    return GF_OK;
}

gf_status gf_forward_noalloc(gf_plan *p, const void *rho, void *d, int batch, void *hip_stream)
{
    if (!p || !rho || !d) return fail(GF_EINVAL, "NULL argument");
    if (batch < 1) return fail(GF_EINVAL, "batch must be >= 1");
    const size_t need = p->ws_bytes(GF_OP_FORWARD, batch);
    if (need > kScratchBytes)
        return fail(GF_EBUSY, "batch %d needs %zu bytes of workspace, beyond the %zu-byte fixed scratch", batch, need,
                    kScratchBytes);
    int dev = -1;
    gf_status s = hip_check(hipGetDevice(&dev), "current device");
    if (s != GF_OK) return s;
    if (dev != p->device) return fail(GF_EINVAL, "current device %d is not the plan's device %d", dev, p->device);
    void *ws = nullptr;
    if ((s = scratch_address(dev, &ws)) != GF_OK) return s;
    return gf_forward(p, rho, d, batch, ws, kScratchBytes, hip_stream);
}

gf_status gf_adjoint(gf_plan *p, const void *r, void *g, int batch, void *workspace,
                     size_t workspace_bytes, void *hip_stream)
{
    if (!p || !r || !g) return fail(GF_EINVAL, "NULL argument");
    if (batch < 1) return fail(GF_EINVAL, "batch must be >= 1");
    gf_status s = check_align(p, r, g);
    if (s != GF_OK) return s;
    s = pick_ws(p, GF_OP_ADJOINT, batch, workspace, workspace_bytes);
    if (s != GF_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    int S, lps;
    p->adj_split(batch, &S, &lps);
    gf::NyqSplit nq{nullptr, 0, 0};
    p->nyq_split(&nq.Sny, &nq.lps_ny);
    // levels in chunks of Tc: per level its residual's row transform and
    // column passes into its own layer-column slabs (one per component
    // group); the inverse row pass sums a chunk's slabs and adds the chunk
    // to g after the first
    const int Tc = p->adj_chunk();
    const size_t rstride = (size_t)batch * p->fwd_slots() * p->M * p->ldc;
    const size_t gstride = (size_t)batch * p->nz * p->M * p->ldc;
    const size_t plane = (size_t)p->nx * p->ny;
    char *R = (char *)workspace;
    char *Gt = R + p->celem() * (size_t)Tc * rstride;
    gf::RowCombo ident{};
    ident.identity = 1;
    const double scale = kGrav / ((double)p->py * p->M);
    const gf::NyqSplit none{nullptr, 0, 0};
    mark(p, GF_OP_ADJOINT, 0, st);
    if (p->levels_toeplitz()) {
        // per chunk of levels: the residuals' row transforms (one launch per
        // level), their column spectra, and the depth products of every group
        // summed into the layer spectra; then the inverse column transforms
        // and rows once
        const int tcm = p->toep_chunk();
        const size_t rs = p->col_slab_bytes(), ss = p->sp_slab_bytes();
        char *Rl = (char *)workspace;
        char *Xr = Rl + rs * (size_t)batch * tcm * p->n_spec;
        char *Gh = Xr + ss * (size_t)batch * tcm * p->n_spec;
        char *Gc = Gh + ss * (size_t)batch * p->nz;
        for (int t0 = 0; t0 < p->nt; t0 += tcm) {
            const int tc = std::min(tcm, p->nt - t0);
            const int slots = tc * p->n_spec;
            // the row transforms of every level of the chunk in one launch per
            // model (levels are consecutive items of n_out planes in r and of
            // n_spec slabs in Rl); one launch for all models when the chunk is
            // every level
            const int nitems = tc == p->nt ? batch * tc : tc;
            for (int b0 = 0; b0 < batch; b0 += nitems / tc)
                if (gf::launch_row_r2c(p->fp64(), p->px,
                                       (const char *)r + p->elem() * ((size_t)b0 * p->nt + t0) * p->n_out * plane, p->nx,
                                       p->nx, p->ny, p->ldc, p->n_spec, p->n_out, nitems, p->in_combo,
                                       Rl + rs * (size_t)b0 * slots, p->tw, p->twlog, st) != 0)
                    return fail(GF_EDEVICE, "row transform launch: %s", hipGetErrorString(hipGetLastError()));
            if (t0 == 0) mark(p, GF_OP_ADJOINT, 1, st);
            if (gf::launch_col_spectra(p->fp64(), p->py, Rl, Xr, batch, slots, p->M, p->ny, p->ldc, p->tw, p->twlog,
                                       st) != 0)
                return fail(GF_EDEVICE, "column spectra launch: %s", hipGetErrorString(hipGetLastError()));
            for (int gr = 0; gr < p->ngrp; ++gr) {
                const char *Xg = Xr + ss * (size_t)p->grp_c0[gr];
                const int e = p->zdepth
                                  ? gf::launch_levelz_adjoint(Xg, p->kz_group(gr), Gh, batch, p->nz, t0, tc,
                                                              p->nt, p->U, p->QP, p->grp_cs[gr], p->n_spec,
                                                              p->grp_bits(p->imag_mask, gr),
                                                              p->grp_bits(p->yodd_mask, gr), t0 > 0 || gr > 0, p->tw,
                                                              p->twlog, st)
                                  : gf::launch_levels_adjoint(p->fp64(), p->py, Xg, p->spec_window(gr, t0), Gh, batch,
                                                              p->nz, tc, p->M, p->grp_cs[gr], p->n_spec,
                                                              p->grp_bits(p->imag_mask, gr),
                                                              p->grp_bits(p->yodd_mask, gr), t0 > 0 || gr > 0, st);
                if (e != 0) return fail(GF_EDEVICE, "depth product launch: %s", hipGetErrorString(hipGetLastError()));
            }
        }
        if (gf::launch_col_inverse(p->fp64(), p->py, Gh, Gc, batch, p->nz, p->M, p->ny, p->ldc, p->tw, p->twlog, st) != 0)
            return fail(GF_EDEVICE, "inverse column launch: %s", hipGetErrorString(hipGetLastError()));
        mark(p, GF_OP_ADJOINT, 2, st);
        if (gf::launch_row_c2r(p->fp64(), p->px, Gc, (long)batch * p->nz * p->M * p->ldc, 1, p->nz, p->ny, p->ldc,
                               p->nz, batch, ident, none, g, p->nx, scale, p->tw, p->twlog, st, 0, false) != 0)
            return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
        mark(p, GF_OP_ADJOINT, 3, st);
        return GF_OK;
    }
    if (p->levels_blocked()) {
        // passes of up to levels_per_pass() levels: one row transform of the
        // pass's residual planes into level-major slots, one column pass
        // into the pass's layer slab
        const int per = p->levels_per_pass(), npass = p->adj_passes();
        for (int q0 = 0; q0 < npass; q0 += Tc) {
            const int qc = std::min(Tc, npass - q0);
            for (int jq = 0; jq < qc; ++jq) {
                const int t0 = (q0 + jq) * per;
                const int nlev = std::min(per, p->nt - t0);
                gf::RowCombo cmb{};
                for (int j = 0; j < nlev; ++j)
                    for (int sl = 0; sl < p->n_spec; ++sl) {
                        const int k = j * p->n_spec + sl;
                        cmb.nterm[k] = p->in_combo.nterm[sl];
                        for (int i = 0; i < p->in_combo.nterm[sl]; ++i) {
                            cmb.src[k][i] = j * p->n_out + p->in_combo.src[sl][i];
                            cmb.w[k][i] = p->in_combo.w[sl][i];
                        }
                    }
                char *Rq = R + p->celem() * (size_t)jq * rstride;
                if (gf::launch_row_r2c(p->fp64(), p->px, (const char *)r + p->elem() * (size_t)t0 * p->n_out * plane,
                                       p->nx, p->nx, p->ny, p->ldc, nlev * p->n_spec, p->nt * p->n_out, batch, cmb,
                                       Rq, p->tw, p->twlog, st) != 0)
                    return fail(GF_EDEVICE, "row transform launch: %s", hipGetErrorString(hipGetLastError()));
                if (q0 + jq == 0) mark(p, GF_OP_ADJOINT, 1, st);
                if (gf::launch_col_adjoint_levels(p->fp64(), p->py, Rq, p->spec_window(0, t0),
                                                  Gt + p->celem() * (size_t)jq * gstride, batch, p->nz, p->M, p->ny,
                                                  p->ldc, p->n_spec, nlev, S, lps, nq, p->imag_mask, p->yodd_mask,
                                                  p->tw, p->twlog, st) != 0)
                    return fail(GF_EDEVICE, "column pass launch: %s", hipGetErrorString(hipGetLastError()));
            }
            if (q0 + qc == npass) mark(p, GF_OP_ADJOINT, 2, st);
            if (gf::launch_row_c2r(p->fp64(), p->px, Gt, (long)gstride, qc, p->nz, p->ny, p->ldc, p->nz, batch, ident,
                                   none, g, p->nx, scale, p->tw, p->twlog, st, 0, q0 > 0) != 0)
                return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
        }
        mark(p, GF_OP_ADJOINT, 3, st);
        return GF_OK;
    }
    for (int t0 = 0; t0 < p->nt; t0 += Tc) {
        const int tc = std::min(Tc, p->nt - t0);
        for (int j = 0; j < tc; ++j) {
            const int t = t0 + j;
            char *Rj = R + p->celem() * (size_t)j * rstride;
            if (gf::launch_row_r2c(p->fp64(), p->px, (const char *)r + p->elem() * (size_t)t * p->n_out * plane, p->nx,
                                   p->nx, p->ny, p->ldc, p->n_spec, p->nt * p->n_out, batch, p->in_combo, Rj, p->tw,
                                   p->twlog, st) != 0)
                return fail(GF_EDEVICE, "row transform launch: %s", hipGetErrorString(hipGetLastError()));
            if (t == 0) mark(p, GF_OP_ADJOINT, 1, st);
            for (int gr = 0; gr < p->ngrp; ++gr) {
                const int c0 = p->grp_c0[gr];
                if (gf::launch_col_adjoint(p->fp64(), p->py, Rj + p->celem() * (size_t)c0 * p->M * p->ldc,
                                           p->spec_window(gr, t), Gt + p->celem() * (size_t)(j * p->ngrp + gr) * gstride,
                                           batch, p->nz, p->M, p->ny, p->ldc, p->grp_cs[gr], p->n_spec, S, lps, nq,
                                           p->grp_bits(p->imag_mask, gr), p->grp_bits(p->yodd_mask, gr), p->tw,
                                           p->twlog, st) != 0)
                    return fail(GF_EDEVICE, "column pass launch: %s", hipGetErrorString(hipGetLastError()));
            }
        }
        if (t0 + tc == p->nt) mark(p, GF_OP_ADJOINT, 2, st);
        if (gf::launch_row_c2r(p->fp64(), p->px, Gt, (long)gstride, tc * p->ngrp, p->nz, p->ny, p->ldc, p->nz, batch,
                               ident, none, g, p->nx, scale, p->tw, p->twlog, st, 0, t0 > 0) != 0)
            return fail(GF_EDEVICE, "inverse row transform launch: %s", hipGetErrorString(hipGetLastError()));
    }
    mark(p, GF_OP_ADJOINT, 3, st);
    return GF_OK;
}

gf_status gf_plan_set_timing(gf_plan *p, int enable)
{
    if (!p) return fail(GF_EINVAL, "NULL plan");
    if (enable && !p->ev[0][0]) {
        for (int o = 0; o < 2; ++o)
            for (int i = 0; i < 4; ++i) {
                gf_status s = hip_check(hipEventCreate(&p->ev[o][i]), "event");
                if (s != GF_OK) return s;
            }
    }
    p->timing = enable != 0;
    return GF_OK;
}

gf_status gf_plan_last_pass_ms(gf_plan *p, int op, double ms[3])
{
    if (!p || !ms) return fail(GF_EINVAL, "NULL argument");
    if (op != GF_OP_FORWARD && op != GF_OP_ADJOINT) return fail(GF_EINVAL, "bad op %d", op);
    if (!p->ev_recorded[op]) return fail(GF_EINVAL, "no timed call of this op yet");
    gf_status s = hip_check(hipEventSynchronize(p->ev[op][3]), "event sync");
    if (s != GF_OK) return s;
    for (int i = 0; i < 3; ++i) {
        float v = 0;
        if ((s = hip_check(hipEventElapsedTime(&v, p->ev[op][i], p->ev[op][i + 1]), "elapsed")) != GF_OK) return s;
        ms[i] = v;
    }
    return GF_OK;
}

gf_status gf_debug_kernel_table(const gf_plan *p, int n, double *host_out)
{
    if (!p || !host_out) return fail(GF_EINVAL, "NULL argument");
    if (n < 0 || n >= p->nzs) return fail(GF_EINVAL, "layer %d out of range", n);
    const size_t field = (size_t)p->py * p->px;
    DevBuf E;
    gf_status s;
    if ((s = hip_check(dev_malloc((void **)&E.p, field * 8 * sizeof(double)), "debug field")) != GF_OK) return s;
    if ((s = hip_check(hipMemset(E.p, 0, field * 8 * sizeof(double)), "memset")) != GF_OK) return s;
    const int codes[8] = {0, 1, 2, 3, 4, 5, 7, 8};
    if (gf::launch_kgen_field(E.p, 1, n, 6, codes, kgen_geom(p), make_rules(), nullptr) != 0 ||
        gf::launch_kgen_field((double *)E.p + 6 * field, 1, n, 2, codes + 6, kgen_geom(p), make_rules(), nullptr) != 0)
        return fail(GF_EDEVICE, "kernel table launch failed");
    std::vector<double> h(field * 8);
    if ((s = hip_check(hipMemcpy(h.data(), E.p, h.size() * sizeof(double), hipMemcpyDeviceToHost), "copy")) != GF_OK)
        return s;
    const int na = 2 * p->nx - 1, nb = 2 * p->ny - 1;
    for (int b = -(p->ny - 1); b <= p->ny - 1; ++b)
        for (int a = -(p->nx - 1); a <= p->nx - 1; ++a) {
            const size_t src = (size_t)((b + p->py) % p->py) * p->px + (size_t)((a + p->px) % p->px);
            const size_t dst = (size_t)(b + p->ny - 1) * na + (size_t)(a + p->nx - 1);
            double v[8];
            for (int c = 0; c < 8; ++c) v[c] = kGrav * h[(size_t)c * field + src];
            for (int c = 0; c < 6; ++c) host_out[(size_t)c * na * nb + dst] = v[c];
            host_out[(size_t)6 * na * nb + dst] = -(v[1] + v[4]);
            host_out[(size_t)7 * na * nb + dst] = v[6];
            host_out[(size_t)8 * na * nb + dst] = v[7];
        }
    return GF_OK;
}

gf_status gf_debug_spectrum(const gf_plan *p, unsigned component, int n, double *host_out)
{
    if (!p || !host_out) return fail(GF_EINVAL, "NULL argument");
    if (n < 0 || n >= p->nzs) return fail(GF_EINVAL, "layer %d out of range", n);
    int code = -1;
    for (int c = 0; c < gf::kMaxOut; ++c)
        if (c != 6 && component == (1u << c)) code = c;
    const int slot_all = code >= 0 ? p->slot_of(code) : -1;
    if (slot_all < 0) return fail(GF_EINVAL, "component 0x%x has no resident spectrum", component);
    const int gr = slot_all / p->gmax, slot = slot_all - p->grp_c0[gr], cs = p->grp_cs[gr];
    // group layout [n][row][slot][QP], rows in the order kx = 0, Px/2, 1, ..., Px/2-1
    const size_t layer = (size_t)p->U * cs * p->QP;
    std::vector<double> lay(layer);
    gf_status s;
    if (p->fp64()) {
        if ((s = hip_check(hipMemcpy(lay.data(), (const double *)p->spec_group(gr) + (size_t)n * layer,
                                     layer * sizeof(double), hipMemcpyDeviceToHost), "copy")) != GF_OK)
            return s;
    } else {
        std::vector<float> tmp(layer);
        if ((s = hip_check(hipMemcpy(tmp.data(), (const float *)p->spec_group(gr) + (size_t)n * layer,
                                     layer * sizeof(float), hipMemcpyDeviceToHost), "copy")) != GF_OK)
            return s;
        for (size_t i = 0; i < layer; ++i) lay[i] = tmp[i];
    }
    for (int kx = 0; kx <= p->M; ++kx) {
        const int row = kx == 0 ? 0 : (kx == p->M ? 1 : kx + 1);
        for (int ky = 0; ky < p->Q; ++ky)
            host_out[(size_t)kx * p->Q + ky] =
                lay[((size_t)row * cs + slot) * p->QP + gf::spec_position(p->fp64(), p->py, ky)];
    }
    return GF_OK;
}

}  // extern "C"
