// Host-side launchers of the HIP kernels, shared by the plan code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace gf {

// Most output components of one plan (gz, the six tensor components, gx, gy)
// and most spectra one column-pass launch carries; plans with more resident
// spectra run the column pass once per group of at most kColMaxSpec (or of
// three or one where the transform length leaves less LDS).
constexpr int kMaxOut = 9;
constexpr int kColMaxSpec = 6;

// How a slab of rows is formed from source slabs: slab s of batch item b is
// sum_i w[s][i] * src_slab(b, src[s][i]).  identity: slab s reads source s.
struct RowCombo {
    int identity;
    int nterm[kMaxOut];
    int src[kMaxOut][2];
    double w[kMaxOut][2];
};

// Layer chunks of the real Nyquist unit (kx = px/2) when the column passes
// run it apart from the main units (col_nyquist_apart): Sny chunks of lps_ny
// layers; the forward pass writes its partial columns to
// Dny[Sny][B][Ct][ldc] (real values), summed by the inverse row pass.
struct NyqSplit {
    void *Dny;
    int Sny, lps_ny;
};

// Gauss-Legendre rules on [-1,1] of orders 6, 4 and 3 (in that order).
struct GLRules {
    double x[13];
    double w[13];
};

struct KgenGeom {
    int nx, ny, px, py;
    double dx, dy, h;
    const double *zedge;  // device, nz + 1 layer-edge depths: layer n spans [zedge[n], zedge[n+1]]
    double t_analytic;   // closed form below this many half-diagonals
    double t_gl6;        // 6^3 rule below this, 4^3 below t_gl4, 3^3 beyond
    double t_gl4;
};

// Forward row transform (real rows of length <= px -> px/2 packed column
// units, written transposed as out[slab][u][row] with leading dimension ldc).
//   in       base of source rows; row (b, src, y) at in + ((b*src_per_b + src)*rows + y)*row_len
//   lin      nonzero entries per row (<= px); the rest of each row is zero
//   rows     rows per slab; nsub slabs per batch item; nbatch items
//   out_bslabs  slabs between batch items of out (0: nsub, packed)
int launch_row_r2c(bool fp64, int px, const void *in, long row_len, int lin, int rows, int ldc,
                   int nsub, int src_per_b, int nbatch, const RowCombo &cmb, void *out, const void *tw,
                   int twlog, hipStream_t st, long out_bslabs = 0);

// Inverse row transform: X(b,o,y)[u] = sum_split sum_i w[o][i] D[split][b][src[o][i]][u][y],
// then real rows of length px, of which the first nx_out are written, times
// `scale`, to out + b*out_bstride + (o*rows + y)*nx_out (out_bstride 0: the
// items are packed, nsub*rows*nx_out apart), or added to what is there when
// `accumulate`.  With nq.Sny > 0 the imaginary field of packed unit 0 (the
// Nyquist bin) is instead sum_chunk sum_i w[o][i] Dny[chunk][b][src[o][i]][y].
int launch_row_c2r(bool fp64, int px, const void *D, long split_stride, int nsplit, int nsrc,
                   int rows, int ldc, int nsub, int nbatch, const RowCombo &cmb, const NyqSplit &nq,
                   void *out, int nx_out, double scale, const void *tw, int twlog, hipStream_t st,
                   long out_bstride = 0, bool accumulate = false);

// Column data are stored per slab as [unit][y] with M = px/2 units and a
// leading dimension ldc >= ny (even, so that columns are 16-byte aligned): unit u
// holds x-bin kx = u for u >= 1, and unit 0 packs the real-valued bins
// kx = 0 (real part) and kx = px/2 (imaginary part).  Spectra are stored
// [Cs][nz][M+1][py/2+1] (quarter plane, one real per frequency).
//
// Whether the column passes of transform length py run the Nyquist unit
// apart from the px/2 main units (else all px/2 + 1 virtual units share the
// layer split and the Nyquist results go to the packed unit 0 of D).
bool col_nyquist_apart(int py);

// Column pass of the forward operator: per column unit u and model b, for
// each layer n of the split: FFT along y, multiply by conj(K^_{c,n}) and
// accumulate over n; then inverse FFT per component.  spec holds Cs
// (<= kColMaxSpec) components; D (and nq.Dny) are laid out with a slot
// stride of Ct >= Cs components, the caller offsetting them to the group's
// first slot.
int launch_col_forward(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz,
                       int M, int ny, int ldc, int Cs, int Ct, int nsplit, int lps, const NyqSplit &nq,
                       unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st);

// Column pass of the adjoint: FFT of the Cs residual columns, then per layer
// sum_c K^_{c,n} r^_c and an inverse FFT.  R is laid out with a slot stride
// of Ct >= Cs components (offset by the caller to the group's first slot).
int launch_col_adjoint(bool fp64, int py, const void *R, const void *spec, void *Gout, int B,
                       int nz, int M, int ny, int ldc, int Cs, int Ct, int nsplit, int lps, const NyqSplit &nq,
                       unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st);

// Forward column pass of nlev observation levels at once for Cs <= 3
// spectra (nlev * Cs <= 6): level j sums spectral layers n + j from `spec`
// over model layers n; D and nq.Dny hold nlev * Cs slots (level-major).
// Only where the transform length runs in the wave split and its buffers fit
// in LDS (col_levels_supported).
int launch_col_forward_levels(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz, int M,
                              int ny, int ldc, int Cs, int nlev, int nsplit, int lps, const NyqSplit &nq,
                              unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st);
// Adjoint column pass of nlev observation levels at once: R holds the
// pass's nlev * Cs residual slots (level-major), Gout one layer-column slab.
int launch_col_adjoint_levels(bool fp64, int py, const void *R, const void *spec, void *Gout, int B, int nz, int M,
                              int ny, int ldc, int Cs, int nlev, int nsplit, int lps, const NyqSplit &nq,
                              unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st);
bool col_levels_supported(bool fp64, int py);

// Observation levels as a Toeplitz product in depth.  A column's spectrum
// is two rows of QP values (row 0: ky = q, row 1: ky = py - q, both at the
// resident position of q); a slab is [M+1 rows][2][QP] complex.
// Spectra X[b*nsrc + s] of the columns of R[b*nsrc + s] (slabs [M][ldc]).
int launch_col_spectra(bool fp64, int py, const void *R, void *X, int B, int nsrc, int M, int ny, int ldc,
                       const void *tw, int twlog, hipStream_t st);
// The inverse: columns D[b*nsrc + s] (y < ny) from the spectra X[b*nsrc + s].
int launch_col_inverse(bool fp64, int py, const void *X, void *D, int B, int nsrc, int M, int ny, int ldc,
                       const void *tw, int twlog, hipStream_t st);
// Whether the two above exist for transform length py (the wave-split lengths).
bool col_spectra_supported(int py);
// Dh[b][o][c] = sum_n conj(K^_{c,o+n}) X[b][n] for o < nlev, n < nz; spec is
// the window of nz + nlev - 1 spectral layers of one group of Cs spectra;
// Dh holds Ct slots per level (offset by the caller to the group's first).
int launch_levels_forward(bool fp64, int py, const void *X, const void *spec, void *Dh, int B, int nz, int nlev, int M,
                          int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, hipStream_t st);
// Gh[b][n] (+)= sum_c sum_t K^_{c,n+t} Rh[b][t][c] for n < nz, t < nlev; Rh holds
// Ct slots per level (offset to the group's first), Gh is added to when accumulate.
int launch_levels_adjoint(bool fp64, int py, const void *Rh, const void *spec, void *Gh, int B, int nz, int nlev, int M,
                          int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, bool accumulate, hipStream_t st);

// Observation levels through a transform in depth of length 256 (FP64
// plans): plan-time Kz[row][c][j][QP] (complex, j <= 128) of a group's window
// of nwin <= 256 spectral layers, and the forward / adjoint of a chunk of
// levels [t0, t0 + tc) of nt, in the layouts of launch_levels_forward /
// launch_levels_adjoint (Kz of the group instead of its spectra window;
// t0 absolute).
bool levelz_supported(int nwin);
size_t levelz_values(int U1, int Cs, int QP);
int launch_levelz_kgen(const void *spec, void *kz, int nwin, int U1, int Cs, int QP, const void *tw64, int twlog,
                       hipStream_t st);
int launch_levelz_forward(const void *X, const void *kz, void *Dh, int B, int nz, int t0, int tc, int nt, int U1,
                          int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog,
                          hipStream_t st);
int launch_levelz_adjoint(const void *Rh, const void *kz, void *Gh, int B, int nz, int t0, int tc, int nt, int U1,
                          int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, bool accumulate,
                          const void *tw, int twlog, hipStream_t st);

// Plan time: column FFT of the row-transformed kernel fields and extraction
// of the quarter-plane spectrum into spec[Cs][nz][M+1][py/2+1] (float or double).
int launch_col_kgen(bool out_fp64, int py, const void *Rk, void *spec, int nl, int n0, int Cs,
                    int nz, int M, unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog,
                    hipStream_t st);

// Plan time: kernel table of layers [n0, n0+nl) for the Cs components in
// codes[], written into zeroed circulant fields E[nl][Cs][py][px] (double).
int launch_kgen_field(void *E, int nl, int n0, int Cs, const int *codes, const KgenGeom &g,
                      const GLRules &gl, hipStream_t st);

// Upper bound of concurrently resident workgroups of the forward column pass
// (for choosing the layer split).
int col_forward_capacity(bool fp64, int py, int Cs, int B);
int col_forward_groups(bool fp64, int py);

// Largest dynamic LDS allocation a workgroup may request on the current
// device (bytes).
size_t lds_limit();

// Padded length (values) of one resident spectrum row for transform length py.
int spec_row_pitch(bool fp64, int py);

// Position of frequency ky in [0, py/2] within a resident spectrum row of
// the given precision (the wave-split column passes store rows in
// residue-block order).
int spec_position(bool fp64, int py, int ky);

// Whether the column passes of transform length py with Cs resident
// components fit the device's LDS.
bool col_supported(bool fp64, int py, int Cs);

}  // namespace gf
