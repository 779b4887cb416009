// Observation levels through a transform in depth (eq. 10-11 with the
// survey of Fig. 2a: stations on nt equally spaced planes).
//
// At a horizontal frequency the data of level o and component c is a
// correlation in depth of the layer spectra of the density X[n] with the
// kernel spectra of the layer offsets k[m] (m < nwin = nz + nt - 1):
//     D[o] = f * sum_{n < nz} k[o + n] X[n],   o < nt,
// with f the factor that turns the stored real k into the conjugated
// spectrum (section 2.2: K^ real, or imaginary; odd in y on the mirrored
// row).  With a transform of length L >= nwin no index wraps, so
//     D[o] = f / L * sum_j Kz[j] Xz[j] W^{-j o},
//     Kz[j] = sum_m k[m] W^{j m},  Xz[j] = sum_n X[n] W^{-j n},  W = e^{-2 pi i / L},
// one transform of X per frequency shared by every component and one
// inverse transform per component, instead of nz * nt products per
// component.  The adjoint is the same correlation with the roles of levels
// and layers exchanged, summed over the components before its single
// inverse transform.  Kz is computed at plan time from the resident spectra
// (the real k makes it Hermitian: L/2 + 1 values are stored).
//
// The plan-time transforms are the in-register 256-point wave transform
// (one wave per sequence); those of the apply run 32 lanes per sequence with
// exchanges through LDS (fewer instructions than the wave transform's
// cross-lane moves).  Lengths up to nwin = 256.  FP64
// plans only: the rounding of the transform is relative to the whole depth
// sequence, which in FP32 leaves levels far above the model with about 1e-5
// of their own size (the direct product keeps them at rounding level).
#include "gf_fft.h"
#include "gf_lane.h"
#include "gf_launch.h"

namespace gf {

namespace {

constexpr int kZL = 256;          // depth transform length
constexpr int kZJ = kZL / 2 + 1;  // stored frequencies of the real kernel sequence
constexpr int kZQ = 8;            // positions of a workgroup (one 128-byte line of FP64 complex values)

// Frequency held by slot s of this lane after the forward wave transform.
template <typename T>
__device__ __forceinline__ unsigned zfreq(unsigned lane, int s)
{
    return ws_out_lane<LaneFFT<T>>(lane) + 64u * (unsigned)s;
}

// Multiply by the factor of component c on half h: forward conj(K^) = k, -i k,
// adjoint K^ = k, i k (imaginary components), negated on the mirrored half
// for components odd in y.
template <typename T, bool ADJ>
__device__ __forceinline__ cx<T> zfactor(cx<T> v, bool im, bool neg)
{
    if (im) v = ADJ ? cx<T>{-v.im, v.re} : cx<T>{v.im, -v.re};
    if (neg) v = cx<T>{-v.re, -v.im};
    return v;
}

// Workgroup of 256 threads: kZQ positions (a tile) of one half of one
// spectrum row; sequence g = threadIdx.x / 32 (position g of the tile) is
// one 256-point transform of 32 lanes, eight points a lane (radix 8, 8, 4
// with two exchanges through LDS ordered by waits on the wave's own LDS
// operations).  Tiles are numbered row * ceil(QP / kZQ) + position tile; of
// 16 consecutive workgroups the first eight take half 0 of eight tiles and
// the next eight half 1 of the same tiles, so that the two workgroups that
// read one Kz tile run on one XCD (workgroups are dealt to the eight XCDs in
// turn) close in time.  The workgroup stages its tiles through LDS so that
// global accesses run along the positions (kZQ consecutive values: 128 bytes
// in FP64): the inputs [n][q], Kz of one component [j][q] (rows padded to
// kZQ + 1 values), and the outputs in the inputs' area, which the
// transforms' exchange arrays share between stagings.  Kz is stored per tile
// ([row][c][tile][j][kZQ]), so one component's tile is one contiguous run.
constexpr int kZNT = 32;              // lanes of one transform
constexpr int kZThreads = kZQ * kZNT;
constexpr int kZPPT = kZL / kZNT;     // points a lane
constexpr int kZXP = kZQ + 1;
constexpr int kZKP = kZQ + 1;
template <typename T>
using ZFFT = BlockFFT<T, kZL, kZNT, 8, true, true, true>;

__host__ __device__ inline int zqtiles(int QP) { return (QP + kZQ - 1) / kZQ; }

struct ZTile {
    unsigned row, tile, q0, g, h, t;
    bool valid, active;
};

__device__ __forceinline__ ZTile ztile(int QP, int ntile)
{
    const unsigned qtiles = (unsigned)zqtiles(QP), bx = blockIdx.x;
    ZTile z;
    z.g = threadIdx.x / kZNT;
    z.t = threadIdx.x % kZNT;
    z.h = (bx >> 3) & 1u;
    z.tile = (bx >> 4) * 8u + (bx & 7u);
    z.valid = z.tile < (unsigned)ntile;
    z.row = z.tile / qtiles;
    z.q0 = (z.tile % qtiles) * kZQ;
    z.active = z.q0 + z.g < (unsigned)QP;
    return z;
}

// LDS of a workgroup (T words): the transforms' stage twiddles, Kz of one
// component, and the area of the staged tiles / exchange arrays.
template <typename T>
struct ZLds {
    static constexpr int STW = (2 * ZFFT<T>::stw_entries() + 1) / 2 * 2;
    static constexpr int KS = 2 * kZJ * kZKP;
    static size_t area_words(int nrows)
    {
        const size_t tiles = (size_t)nrows * kZXP * 2, xch = (size_t)kZQ * ZFFT<T>::lds_group_words();
        return tiles > xch ? tiles : xch;
    }
    static size_t bytes(int nrows) { return (STW + KS + area_words(nrows)) * sizeof(T); }
};

template <typename T>
size_t levelz_lds_bytes(int nrows)
{
    return ZLds<T>::bytes(nrows);
}

// Staged element of a [rows][kZQ] tile of half h (rows <= L): row,
// position; positions past QP give zero.  All of a thread's loads are issued
// before the first is used (addresses clamped into the tile, values selected
// afterwards).
template <typename T>
__device__ __forceinline__ void stage_tile(cx<T> *dst, const cx<T> *__restrict__ src, size_t slab0, size_t slab_step,
                                           int nrows, size_t xslab, unsigned row, unsigned h, unsigned q0, int QP)
{
    constexpr int PER = kZL * kZQ / kZThreads;
    const unsigned qq = threadIdx.x % kZQ;
    const bool qok = q0 + qq < (unsigned)QP;
    const cx<T> *base = src + slab0 * xslab + ((size_t)row * 2 + h) * QP + (qok ? q0 + qq : 0u);
    cx<T> v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int r = (int)(threadIdx.x / kZQ) + i * (kZThreads / kZQ);
        v[i] = base[(size_t)(r < nrows ? r : 0) * slab_step * xslab];
    }
    // rows past nrows go to the padding slot of row 0 (never read): stores
    // without branches keep v in registers
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int r = (int)(threadIdx.x / kZQ) + i * (kZThreads / kZQ);
        dst[r < nrows ? r * kZXP + (int)qq : kZQ] = qok ? v[i] : cx<T>{T(0), T(0)};
    }
}

// Stores the staged [rows][kZQ] tile of half h to dst (slab r at
// dst + r * slab_step * xslab), added to what is there when accumulate.
template <typename T>
__device__ __forceinline__ void store_tile(cx<T> *__restrict__ dst, const cx<T> *src, size_t slab0, size_t slab_step,
                                           int nrows, size_t xslab, unsigned row, unsigned h, unsigned q0, int QP,
                                           bool accumulate)
{
    const unsigned qq = threadIdx.x % kZQ;
    if (q0 + qq >= (unsigned)QP) return;
    cx<T> *base = dst + slab0 * xslab + ((size_t)row * 2 + h) * QP + q0 + qq;
    for (int r = (int)(threadIdx.x / kZQ); r < nrows; r += kZThreads / kZQ) {
        cx<T> *d = base + (size_t)r * slab_step * xslab;
        cx<T> v = src[r * kZXP + qq];
        if (accumulate) v = add(*d, v);
        *d = v;
    }
}

// Kz of one component for this tile ([j][kZQ], contiguous): each thread's
// elements (four whole rounds of the workgroup, then the last kZQ values by
// the first threads), loaded into registers and put into LDS (rows padded).
// Named members rather than an array: the values live across the component
// loop, and an array there was kept in scratch memory.
template <typename T>
struct KzShare {
    static_assert(kZJ * kZQ == 4 * kZThreads + kZQ, "four rounds and kZQ values");
    cx<T> v0, v1, v2, v3, tail;
    __device__ __forceinline__ void load(const cx<T> *__restrict__ kzt)
    {
        v0 = kzt[threadIdx.x];
        v1 = kzt[threadIdx.x + kZThreads];
        v2 = kzt[threadIdx.x + 2 * kZThreads];
        v3 = kzt[threadIdx.x + 3 * kZThreads];
        tail = kzt[4 * kZThreads + threadIdx.x % kZQ];
    }
    __device__ __forceinline__ static void put1(cx<T> *ks, int e, cx<T> v) { ks[(e / kZQ) * kZKP + e % kZQ] = v; }
    __device__ __forceinline__ void put(cx<T> *ks) const
    {
        put1(ks, (int)threadIdx.x, v0);
        put1(ks, (int)threadIdx.x + kZThreads, v1);
        put1(ks, (int)threadIdx.x + 2 * kZThreads, v2);
        put1(ks, (int)threadIdx.x + 3 * kZThreads, v3);
        if (threadIdx.x < (unsigned)kZQ) ks[(kZJ - 1) * kZKP + threadIdx.x] = tail;
    }
};

// Kz of frequency j at position column qi from the staged tile.
template <typename T>
__device__ __forceinline__ cx<T> kz_lds(const cx<T> *ks, unsigned j, unsigned qi)
{
    if (j < (unsigned)kZJ) return ks[j * kZKP + qi];
    return conjg(ks[(kZL - j) * kZKP + qi]);
}

// register order of the transform's output -> its input order
template <typename T>
__device__ __forceinline__ void zout_to_in(cx<T> (&v)[kZPPT])
{
    cx<T> tmp[kZPPT];
#pragma unroll
    for (int s = 0; s < kZPPT; ++s) tmp[s] = v[s];
#pragma unroll
    for (int s = 0; s < kZPPT; ++s)
#pragma unroll
        for (int q = 0; q < kZPPT; ++q)
            if (ZFFT<T>::elem_out(q) == ZFFT<T>::elem_in(s)) v[s] = tmp[q];
}

// Plan time: Kz[row][c][tile][j][q mod kZQ], j <= L/2, of the window of nwin
// spectral layers spec[m][row][c][q] (real).  One wave per (row, c, q); 16
// consecutive positions a workgroup.
template <typename TO>
__global__ void __launch_bounds__(1024) levelz_kgen_kernel(const TO *__restrict__ spec, cx<TO> *__restrict__ kz,
                                                          int nwin, int U1, int Cs, int QP,
                                                          const cx<double> *__restrict__ tw, int twlog)
{
    const unsigned lane = threadIdx.x & 63u;
    const long nseq = (long)U1 * Cs * QP;
    const long wid = (long)blockIdx.x * 16 + (threadIdx.x >> 6);
    if (wid >= nseq) return;   // whole waves: the transform has no workgroup barrier
    const long rc = wid / QP;  // row * Cs + c
    const unsigned q = (unsigned)(wid % QP);
    cx<TO> *kzt = kz + ((size_t)rc * zqtiles(QP) + q / kZQ) * kZJ * kZQ + q % kZQ;
    const size_t kstride = (size_t)U1 * Cs * QP;
    cx<double> v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int m = (int)lane + 64 * s;
        v[s] = cx<double>{m < nwin ? (double)spec[(size_t)m * kstride + (size_t)rc * QP + q] : 0.0, 0.0};
    }
    cx<double> t[9];
    lane_twiddles<false>(t, tw, twlog, lane);
    lane_fft<false>(v, lane, t);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const unsigned j = zfreq<double>(lane, s);
        if (j < (unsigned)kZJ) kzt[(size_t)j * kZQ] = cx<TO>{(TO)v[s].re, (TO)v[s].im};
    }
}

// Forward: Dh[b][o - t0][c] for the chunk of levels o in [t0, t0 + tc), of
// every component of the group (Kz of the group: [U1][Cs][L/2+1][QP]); X is
// [B][nz][U1][2][QP], Dh [B][tc][Ct][U1][2][QP] (offset by the caller to the
// group's first slot).  The next component's Kz is loaded into registers
// while this one is transformed.
template <typename T>
__global__ void __launch_bounds__(kZThreads) __attribute__((amdgpu_waves_per_eu(3)))
    levelz_forward_kernel(const cx<T> *__restrict__ X, const cx<T> *__restrict__ kz, cx<T> *__restrict__ Dh, int nz,
                          int t0, int tc, int U1, int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask,
                          int ntile, const cx<T> *__restrict__ tw, int twlog)
{
    using F = ZFFT<T>;
    using LD = ZLds<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *stw = reinterpret_cast<T *>(smem_raw);
    cx<T> *ks = reinterpret_cast<cx<T> *>(stw + LD::STW);
    cx<T> *xs = ks + kZJ * kZKP;                                        // tiles, or the exchange arrays
    const ZTile z = ztile(QP, ntile);
    if (!z.valid) return;   // padding workgroups of the last group of 16
    T *xch = reinterpret_cast<T *>(xs) + (size_t)z.g * F::lds_group_words();
    const cx<T> *stp = reinterpret_cast<const cx<T> *>(stw);
    const unsigned b = blockIdx.y;
    const size_t xslab = (size_t)U1 * 2 * QP, kzstep = (size_t)zqtiles(QP) * kZJ * kZQ;
    const cx<T> *kzr = kz + ((size_t)z.row * Cs * zqtiles(QP) + z.q0 / kZQ) * kZJ * kZQ;   // component c at + c kzstep
    F::load_stage_table(stw, tw, twlog, threadIdx.x, kZThreads);
    KzShare<T> kn;
    kn.load(kzr);
    stage_tile(xs, X, (size_t)b * nz, 1, nz, xslab, z.row, z.h, z.q0, QP);
    __syncthreads();
    // conj of the transform of conj(X): sum_n X[n] W^{-j n}, then in input order
    cx<T> y[kZPPT];
#pragma unroll
    for (int s = 0; s < kZPPT; ++s) {
        const int n = (int)z.t + kZNT * F::elem_in(s);
        y[s] = n < nz ? conjg(xs[n * kZXP + z.g]) : cx<T>{T(0), T(0)};
    }
    __syncthreads();   // every sequence has its inputs: the area takes the exchange arrays
    F::template run<false>(y, xch, nullptr, z.t, stp, twlog);
    zout_to_in(y);
#pragma unroll
    for (int s = 0; s < kZPPT; ++s) y[s] = conjg(y[s]);
    const T sc = T(1) / T(kZL);
    for (int c = 0; c < Cs; ++c) {
        kn.put(ks);
        __syncthreads();   // Kz of c staged; every thread is past its stores of the previous outputs
        kn.load(kzr + (size_t)(c + 1 < Cs ? c + 1 : c) * kzstep);   // the next component's (unconditional)
        cx<T> p[kZPPT];
#pragma unroll
        for (int s = 0; s < kZPPT; ++s) p[s] = mul(kz_lds(ks, z.t + (unsigned)(kZNT * F::elem_in(s)), z.g), y[s]);
        F::template run<true>(p, xch, nullptr, z.t, stp, twlog);
        const bool im = (imag_mask >> c) & 1u, neg = z.h && ((yodd_mask >> c) & 1u);
        __syncthreads();   // every sequence is past its exchanges: the area takes the outputs
#pragma unroll
        for (int s = 0; s < kZPPT; ++s) {
            const int o = (int)z.t + kZNT * F::elem_out(s);
            if (o >= t0 && o < t0 + tc) xs[(o - t0) * kZXP + z.g] = zfactor<T, false>(scale(p[s], sc), im, neg);
        }
        __syncthreads();
        store_tile(Dh, xs, (size_t)b * tc * Ct + c, (size_t)Ct, tc, xslab, z.row, z.h, z.q0, QP, false);
    }
}

// Adjoint: Gh[b][n] (+)= sum_c sum_{t in chunk} K^_{c, n + t} Rh[b][t - t0][c]
// for n < nz; Rh is [B][tc][Ct][U1][2][QP] (offset to the group's first slot),
// Gh [B][nz][U1][2][QP].  Per component the inputs of the chunk are staged,
// transformed and multiplied by Kz into the sum; one inverse transform.
template <typename T>
__global__ void __launch_bounds__(kZThreads) __attribute__((amdgpu_waves_per_eu(3)))
    levelz_adjoint_kernel(const cx<T> *__restrict__ Rh, const cx<T> *__restrict__ kz, cx<T> *__restrict__ Gh, int nz,
                          int t0, int tc, int U1, int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask,
                          int accumulate, int ntile, const cx<T> *__restrict__ tw, int twlog)
{
    using F = ZFFT<T>;
    using LD = ZLds<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *stw = reinterpret_cast<T *>(smem_raw);
    cx<T> *ks = reinterpret_cast<cx<T> *>(stw + LD::STW);
    cx<T> *xs = ks + kZJ * kZKP;                                        // tiles, or the exchange arrays
    const ZTile z = ztile(QP, ntile);
    if (!z.valid) return;   // padding workgroups of the last group of 16
    T *xch = reinterpret_cast<T *>(xs) + (size_t)z.g * F::lds_group_words();
    const cx<T> *stp = reinterpret_cast<const cx<T> *>(stw);
    const unsigned b = blockIdx.y;
    const size_t xslab = (size_t)U1 * 2 * QP, kzstep = (size_t)zqtiles(QP) * kZJ * kZQ;
    const cx<T> *kzr = kz + ((size_t)z.row * Cs * zqtiles(QP) + z.q0 / kZQ) * kZJ * kZQ;
    F::load_stage_table(stw, tw, twlog, threadIdx.x, kZThreads);
    cx<T> acc[kZPPT];
#pragma unroll
    for (int s = 0; s < kZPPT; ++s) acc[s] = cx<T>{T(0), T(0)};
    for (int c = 0; c < Cs; ++c) {
        // every sequence is past its exchanges of the previous component (and
        // the stage twiddles are in place)
        __syncthreads();
        {
            KzShare<T> kn;
            kn.load(kzr + (size_t)c * kzstep);
            stage_tile(xs, Rh, (size_t)b * tc * Ct + c, (size_t)Ct, tc, xslab, z.row, z.h, z.q0, QP);
            kn.put(ks);
        }
        __syncthreads();
        const bool im = (imag_mask >> c) & 1u, neg = z.h && ((yodd_mask >> c) & 1u);
        cx<T> y[kZPPT];
#pragma unroll
        for (int s = 0; s < kZPPT; ++s) {
            const int tt = (int)z.t + kZNT * F::elem_in(s);
            y[s] = (tt >= t0 && tt < t0 + tc) ? conjg(zfactor<T, true>(xs[(tt - t0) * kZXP + z.g], im, neg))
                                              : cx<T>{T(0), T(0)};
        }
        __syncthreads();   // every sequence has its inputs: the area takes the exchange arrays
        F::template run<false>(y, xch, nullptr, z.t, stp, twlog);
        zout_to_in(y);
#pragma unroll
        for (int s = 0; s < kZPPT; ++s)
            acc[s] = add(acc[s], mul(kz_lds(ks, z.t + (unsigned)(kZNT * F::elem_in(s)), z.g), conjg(y[s])));
    }
    F::template run<true>(acc, xch, nullptr, z.t, stp, twlog);
    __syncthreads();   // every sequence is past its exchanges: the area takes the outputs
    const T sc = T(1) / T(kZL);
#pragma unroll
    for (int s = 0; s < kZPPT; ++s) {
        const int n = (int)z.t + kZNT * F::elem_out(s);
        if (n < nz) xs[n * kZXP + z.g] = scale(acc[s], sc);
    }
    __syncthreads();
    store_tile(Gh, xs, (size_t)b * nz, 1, nz, xslab, z.row, z.h, z.q0, QP, accumulate != 0);
}

}  // namespace

bool levelz_supported(int nwin) { return nwin >= 1 && nwin <= kZL; }

size_t levelz_values(int U1, int Cs, int QP) { return (size_t)U1 * Cs * zqtiles(QP) * kZJ * kZQ; }

int launch_levelz_kgen(const void *spec, void *kz, int nwin, int U1, int Cs, int QP, const void *tw64, int twlog,
                       hipStream_t st)
{
    if (!levelz_supported(nwin) || U1 < 1 || Cs < 1 || QP < 1 || twlog < 8) return -2;
    const long nseq = (long)U1 * Cs * QP;
    const unsigned nblk = (unsigned)((nseq + 15) / 16);
    hipLaunchKernelGGL(levelz_kgen_kernel<double>, dim3(nblk), dim3(1024), 0, st, (const double *)spec,
                       (cx<double> *)kz, nwin, U1, Cs, QP, (const cx<double> *)tw64, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_levelz_forward(const void *X, const void *kz, void *Dh, int B, int nz, int t0, int tc, int nt, int U1,
                          int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog,
                          hipStream_t st)
{
    if (B < 1 || nz < 1 || tc < 1 || t0 < 0 || t0 + tc > nt || !levelz_supported(nz + nt - 1) || Cs < 1 ||
        Ct < Cs || twlog < 8)
        return -2;
    const int ntile = U1 * zqtiles(QP);
    const dim3 grid((unsigned)(((ntile + 7) / 8) * 16), (unsigned)B);
    const size_t lds = levelz_lds_bytes<double>(nz > tc ? nz : tc);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL(levelz_forward_kernel<double>, grid, dim3(kZThreads), lds, st, (const cx<double> *)X,
                       (const cx<double> *)kz, (cx<double> *)Dh, nz, t0, tc, U1, QP, Cs, Ct, imag_mask, yodd_mask,
                       ntile, (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_levelz_adjoint(const void *Rh, const void *kz, void *Gh, int B, int nz, int t0, int tc, int nt, int U1,
                          int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, bool accumulate,
                          const void *tw, int twlog, hipStream_t st)
{
    if (B < 1 || nz < 1 || tc < 1 || t0 < 0 || t0 + tc > nt || !levelz_supported(nz + nt - 1) || Cs < 1 ||
        Ct < Cs || twlog < 8)
        return -2;
    const int ntile = U1 * zqtiles(QP);
    const dim3 grid((unsigned)(((ntile + 7) / 8) * 16), (unsigned)B);
    const size_t lds = levelz_lds_bytes<double>(nz > tc ? nz : tc);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL(levelz_adjoint_kernel<double>, grid, dim3(kZThreads), lds, st, (const cx<double> *)Rh,
                       (const cx<double> *)kz, (cx<double> *)Gh, nz, t0, tc, U1, QP, Cs, Ct, imag_mask, yodd_mask,
                       accumulate ? 1 : 0, ntile, (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gf
