// Column (y-direction) pass of the 2-D FFT with the per-frequency layer
// reduction between the forward and inverse transforms.
//
// For the forward operator (eq. 21-22: G = [G_11 ... G_1nz], each block
// BTTB) the data spectrum of component c at frequency k is
//     d^_c(k) = sum_n conj(K^_{c,n}(k)) rho^_n(k)
// (d(p) = sum_l K(l-p) rho(l) is a correlation, so the embedded kernel enters
// conjugated).  One group of NT threads owns one column unit u (kx = u) of
// one model: it transforms the layer's column along y, multiplies it by the
// resident quarter-plane spectra and accumulates in registers across the
// layers of its split, then inverse-transforms each component once.  The
// adjoint runs the same steps in transposed roles (no conjugate).
//
// Spectra are stored as one real per frequency on kx in [0,Px/2],
// ky in [0,Py/2]: K^ is purely real (gz, gxx, gxy, gyy) or purely imaginary
// (gxz, gyz), and K^(kx,-ky) = +-K^(kx,ky) with the sign of the component's
// parity in y.
#include "gf_fft.h"
#include "gf_launch.h"

namespace gf {

template <typename T, int N>
struct ColCfg {
    static constexpr int PPT = (sizeof(T) == 4) ? 8 : (N > 2048 ? 8 : 4);
    static constexpr int NT = N / PPT;
    static constexpr int RADIX = PPT;
    using FFT = BlockFFT<T, N, NT, RADIX>;
    static constexpr int W = FFT::lds_words();
    static constexpr int THREADS = NT >= 256 ? NT : 256;
    static constexpr int G = THREADS / NT;          // groups (column units) per workgroup
    static constexpr size_t LDS = (size_t)G * 2 * W * sizeof(T);
};

// reorder registers from the FFT output layout to the FFT input layout
// (both are strided by NT; only the slot order differs)
template <typename F, typename T, int PPT>
__device__ __forceinline__ void out_to_in(cx<T> (&v)[PPT])
{
    cx<T> tmp[PPT];
#pragma unroll
    for (int s = 0; s < PPT; ++s) tmp[s] = v[s];
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            if (F::elem_out(q) == F::elem_in(s)) v[s] = tmp[q];
    }
}

template <typename T, int N, int CMAX>
__global__ void __launch_bounds__((ColCfg<T, N>::THREADS))
    col_forward_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec,
                       cx<T> *__restrict__ D, int B, int nz, int U, int ny, int Cs, int lps,
                       unsigned imag_mask, unsigned yodd_mask, const cx<T> *__restrict__ tw, int twlog)
{
    using C = ColCfg<T, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, W = C::W;
    constexpr int Q = N / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const int g = threadIdx.x / NT;
    const int t = threadIdx.x % NT;
    T *sre = lds + (size_t)g * 2 * W;
    T *sim = sre + W;

    const long gi = (long)blockIdx.x * G + g;
    const bool active = gi < (long)U * B;
    const int u = active ? (int)(gi / B) : 0;
    const int b = active ? (int)(gi % B) : 0;
    const int split = blockIdx.y;
    const int n0 = split * lps;
    const int n1 = min(nz, n0 + lps);

    cx<T> acc[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
#pragma unroll
        for (int s = 0; s < PPT; ++s) acc[c][s] = cx<T>{T(0), T(0)};

    for (int n = n0; n < n1; ++n) {
        cx<T> v[PPT];
        const cx<T> *col = R + (((long)b * nz + n) * U + u) * (long)ny;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const int y = t + NT * F::elem_in(s);
            v[s] = (active && y < ny) ? col[y] : cx<T>{T(0), T(0)};
        }
        F::template run<false>(v, sre, sim, t, tw, twlog);
#pragma unroll
        for (int c = 0; c < CMAX; ++c) {
            if (c < Cs) {
                const T *sp = spec + ((long)(c * nz + n) * U + u) * (long)Q;
                const bool im = (imag_mask >> c) & 1u;
                const bool yo = (yodd_mask >> c) & 1u;
#pragma unroll
                for (int s = 0; s < PPT; ++s) {
                    const int ky = t + NT * F::elem_out(s);
                    const int kq = ky <= N / 2 ? ky : N - ky;
                    T k = active ? sp[kq] : T(0);
                    if (yo && ky > N / 2) k = -k;
                    if (im) {  // conj(i k) v = -i k v
                        acc[c][s].re += k * v[s].im;
                        acc[c][s].im -= k * v[s].re;
                    } else {
                        acc[c][s].re += k * v[s].re;
                        acc[c][s].im += k * v[s].im;
                    }
                }
            }
        }
    }

#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        if (c < Cs) {
            out_to_in<F, T, PPT>(acc[c]);
            F::template run<true>(acc[c], sre, sim, t, tw, twlog);
            if (active) {
                cx<T> *dst = D + ((((long)split * B + b) * Cs + c) * U + u) * (long)ny;
#pragma unroll
                for (int s = 0; s < PPT; ++s) {
                    const int y = t + NT * F::elem_out(s);
                    if (y < ny) dst[y] = acc[c][s];
                }
            }
        }
    }
}

template <typename T, int N, int CMAX>
__global__ void __launch_bounds__((ColCfg<T, N>::THREADS))
    col_adjoint_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec,
                       cx<T> *__restrict__ Gout, int B, int nz, int U, int ny, int Cs, int lps,
                       unsigned imag_mask, unsigned yodd_mask, const cx<T> *__restrict__ tw, int twlog)
{
    using C = ColCfg<T, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, W = C::W;
    constexpr int Q = N / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const int g = threadIdx.x / NT;
    const int t = threadIdx.x % NT;
    T *sre = lds + (size_t)g * 2 * W;
    T *sim = sre + W;

    const long gi = (long)blockIdx.x * G + g;
    const bool active = gi < (long)U * B;
    const int u = active ? (int)(gi / B) : 0;
    const int b = active ? (int)(gi % B) : 0;
    const int split = blockIdx.y;
    const int n0 = split * lps;
    const int n1 = min(nz, n0 + lps);

    cx<T> rh[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        if (c < Cs) {
            const cx<T> *col = R + (((long)b * Cs + c) * U + u) * (long)ny;
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const int y = t + NT * F::elem_in(s);
                rh[c][s] = (active && y < ny) ? col[y] : cx<T>{T(0), T(0)};
            }
            F::template run<false>(rh[c], sre, sim, t, tw, twlog);
        } else {
#pragma unroll
            for (int s = 0; s < PPT; ++s) rh[c][s] = cx<T>{T(0), T(0)};
        }
    }

    for (int n = n0; n < n1; ++n) {
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) v[s] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int c = 0; c < CMAX; ++c) {
            if (c < Cs) {
                const T *sp = spec + ((long)(c * nz + n) * U + u) * (long)Q;
                const bool im = (imag_mask >> c) & 1u;
                const bool yo = (yodd_mask >> c) & 1u;
#pragma unroll
                for (int s = 0; s < PPT; ++s) {
                    const int ky = t + NT * F::elem_out(s);
                    const int kq = ky <= N / 2 ? ky : N - ky;
                    T k = active ? sp[kq] : T(0);
                    if (yo && ky > N / 2) k = -k;
                    if (im) {  // (i k) r
                        v[s].re -= k * rh[c][s].im;
                        v[s].im += k * rh[c][s].re;
                    } else {
                        v[s].re += k * rh[c][s].re;
                        v[s].im += k * rh[c][s].im;
                    }
                }
            }
        }
        out_to_in<F, T, PPT>(v);
        F::template run<true>(v, sre, sim, t, tw, twlog);
        if (active) {
            cx<T> *dst = Gout + (((long)b * nz + n) * U + u) * (long)ny;
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const int y = t + NT * F::elem_out(s);
                if (y < ny) dst[y] = v[s];
            }
        }
    }
}

// Plan time: full-length column FFT of the row-transformed kernel fields
// (double), keeping one real per frequency of the quarter plane.
template <typename TO, int N>
__global__ void __launch_bounds__((ColCfg<double, N>::THREADS))
    col_kgen_kernel(const cx<double> *__restrict__ Rk, TO *__restrict__ spec, int nl, int n0, int Cs,
                    int nz, int U, unsigned imag_mask, const cx<double> *__restrict__ tw, int twlog)
{
    using C = ColCfg<double, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, W = C::W;
    constexpr int Q = N / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const int g = threadIdx.x / NT;
    const int t = threadIdx.x % NT;
    double *sre = lds + (size_t)g * 2 * W;
    double *sim = sre + W;

    const long npair = (long)nl * Cs;
    const long gi = (long)blockIdx.x * G + g;
    const bool active = gi < npair * U;
    const long pair = active ? gi / U : 0;
    const int u = active ? (int)(gi % U) : 0;
    const int c = (int)(pair % Cs);
    const int n = n0 + (int)(pair / Cs);

    cx<double> v[PPT];
    const cx<double> *col = Rk + (pair * U + u) * (long)N;
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int y = t + NT * F::elem_in(s);
        v[s] = active ? col[y] : cx<double>{0.0, 0.0};
    }
    F::template run<false>(v, sre, sim, t, tw, twlog);
    if (active) {
        const bool im = (imag_mask >> c) & 1u;
        TO *dst = spec + ((long)(c * nz + n) * U + u) * (long)Q;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const int ky = t + NT * F::elem_out(s);
            if (ky <= N / 2) dst[ky] = (TO)(im ? v[s].im : v[s].re);
        }
    }
}

template <typename T, int N, int CMAX>
static int run_fwd(const void *R, const void *spec, void *D, int B, int nz, int U, int ny, int Cs,
                   int nsplit, int lps, unsigned imag_mask, unsigned yodd_mask, const void *tw,
                   int twlog, hipStream_t st)
{
    using C = ColCfg<T, N>;
    const long groups = (long)U * B;
    const long nblk = (groups + C::G - 1) / C::G;
    if (C::LDS > lds_limit()) return -3;
    hipLaunchKernelGGL((col_forward_kernel<T, N, CMAX>), dim3((unsigned)nblk, (unsigned)nsplit),
                       dim3(C::THREADS), C::LDS, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)D,
                       B, nz, U, ny, Cs, lps, imag_mask, yodd_mask, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int N, int CMAX>
static int run_adj(const void *R, const void *spec, void *Gout, int B, int nz, int U, int ny, int Cs,
                   int nsplit, int lps, unsigned imag_mask, unsigned yodd_mask, const void *tw,
                   int twlog, hipStream_t st)
{
    using C = ColCfg<T, N>;
    const long groups = (long)U * B;
    const long nblk = (groups + C::G - 1) / C::G;
    if (C::LDS > lds_limit()) return -3;
    hipLaunchKernelGGL((col_adjoint_kernel<T, N, CMAX>), dim3((unsigned)nblk, (unsigned)nsplit),
                       dim3(C::THREADS), C::LDS, st, (const cx<T> *)R, (const T *)spec,
                       (cx<T> *)Gout, B, nz, U, ny, Cs, lps, imag_mask, yodd_mask,
                       (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename TO, int N>
static int run_kgen(const void *Rk, void *spec, int nl, int n0, int Cs, int nz, int U,
                    unsigned imag_mask, const void *tw, int twlog, hipStream_t st)
{
    using C = ColCfg<double, N>;
    const long groups = (long)nl * Cs * U;
    const long nblk = (groups + C::G - 1) / C::G;
    if (C::LDS > lds_limit()) return -3;
    hipLaunchKernelGGL((col_kgen_kernel<TO, N>), dim3((unsigned)nblk), dim3(C::THREADS), C::LDS, st,
                       (const cx<double> *)Rk, (TO *)spec, nl, n0, Cs, nz, U, imag_mask,
                       (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define GF_COL_SIZES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <typename T, int N>
static int fwd_c(int Cs, const void *R, const void *spec, void *D, int B, int nz, int U, int ny,
                 int nsplit, int lps, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs <= 1) return run_fwd<T, N, 1>(R, spec, D, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_fwd<T, N, 3>(R, spec, D, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
    return run_fwd<T, N, 6>(R, spec, D, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
}

template <typename T, int N>
static int adj_c(int Cs, const void *R, const void *spec, void *Gout, int B, int nz, int U, int ny,
                 int nsplit, int lps, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs <= 1) return run_adj<T, N, 1>(R, spec, Gout, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_adj<T, N, 3>(R, spec, Gout, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
    return run_adj<T, N, 6>(R, spec, Gout, B, nz, U, ny, Cs, nsplit, lps, im, yo, tw, twlog, st);
}

int launch_col_forward(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz,
                       int U, int ny, int Cs, int nsplit, int lps, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || Cs > 6) return -2;
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? fwd_c<double, NN>(Cs, R, spec, D, B, nz, U, ny, nsplit, lps, imag_mask,    \
                                        yodd_mask, tw, twlog, st)                                \
                    : fwd_c<float, NN>(Cs, R, spec, D, B, nz, U, ny, nsplit, lps, imag_mask,     \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_adjoint(bool fp64, int py, const void *R, const void *spec, void *Gout, int B,
                       int nz, int U, int ny, int Cs, int nsplit, int lps, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || Cs > 6) return -2;
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? adj_c<double, NN>(Cs, R, spec, Gout, B, nz, U, ny, nsplit, lps, imag_mask, \
                                        yodd_mask, tw, twlog, st)                                \
                    : adj_c<float, NN>(Cs, R, spec, Gout, B, nz, U, ny, nsplit, lps, imag_mask,  \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_kgen(bool out_fp64, int py, const void *Rk, void *spec, int nl, int n0, int Cs,
                    int nz, int U, unsigned imag_mask, const void *tw, int twlog, hipStream_t st)
{
#define CASE(NN)                                                                                  \
    case NN:                                                                                      \
        return out_fp64 ? run_kgen<double, NN>(Rk, spec, nl, n0, Cs, nz, U, imag_mask, tw, twlog, st) \
                        : run_kgen<float, NN>(Rk, spec, nl, n0, Cs, nz, U, imag_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

template <typename T, int N>
static int capacity_of(int Cs)
{
    int nb = 0;
    hipError_t e;
    using C = ColCfg<T, N>;
    if (Cs <= 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 1>, C::THREADS, C::LDS);
    else if (Cs <= 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 3>, C::THREADS, C::LDS);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 6>, C::THREADS, C::LDS);
    if (e != hipSuccess || nb < 1) nb = 1;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    return nb * ncu;
}

int col_forward_capacity(bool fp64, int py, int Cs, int /*B*/)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? capacity_of<double, NN>(Cs) : capacity_of<float, NN>(Cs);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return 256;
    }
#undef CASE
}

size_t lds_limit()
{
    static thread_local int cached_dev = -1;
    static thread_local size_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (dev != cached_dev) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cached = (size_t)v;
        cached_dev = dev;
    }
    return cached;
}

int col_forward_groups(bool fp64, int py)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? ColCfg<double, NN>::G : ColCfg<float, NN>::G;
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return 1;
    }
#undef CASE
}

}  // namespace gf
