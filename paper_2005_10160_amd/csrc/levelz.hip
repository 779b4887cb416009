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
// Every transform is the in-register 256-point wave transform: one wave per
// (spectrum row, half, position) sequence, so lengths up to nwin = 256.  FP64
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

// Workgroup of kZQ waves: kZQ positions of one half of one spectrum row
// (workgroup x index 2 * tile + half, tile = row * ceil(QP / kZQ) + position
// tile, so that the two halves that share Kz are neighbours); wave w takes
// position w.  The workgroup stages its tiles through LDS so that global
// accesses run along the positions (kZQ consecutive values: 128 bytes in
// FP64): the inputs [n][q], Kz of one component [j][q] and the outputs in the
// inputs' area, rows padded to kZQ + 1 values.  Eight waves a workgroup let
// two workgroups share a CU in FP64 (110 registers a lane), one staging while
// the other transforms.
constexpr int kZThreads = 64 * kZQ;
constexpr int kZXP = kZQ + 1;
constexpr int kZKP = kZQ + 1;

struct ZTile {
    unsigned row, q0, h, qi, w, lane;
    bool active;
};

__device__ __forceinline__ ZTile ztile(int QP)
{
    const unsigned qtiles = (unsigned)(QP + kZQ - 1) / kZQ, tile = blockIdx.x >> 1;
    ZTile z;
    z.lane = threadIdx.x & 63u;
    z.w = threadIdx.x >> 6;
    z.row = tile / qtiles;
    z.q0 = (tile % qtiles) * kZQ;
    z.h = blockIdx.x & 1u;
    z.qi = z.w;
    z.active = z.q0 + z.qi < (unsigned)QP;
    return z;
}

template <typename T>
size_t levelz_lds_bytes(int nrows)
{
    return ((size_t)nrows * kZXP + (size_t)kZJ * kZKP) * sizeof(cx<T>);
}

// Staged element e of a [rows][kZQ] tile of half h (rows <= L): row
// e / kZQ, position e % kZQ; positions past QP give zero.  All of a thread's
// loads are issued before the first is used (addresses clamped into the
// tile, values selected afterwards).
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
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int r = (int)(threadIdx.x / kZQ) + i * (kZThreads / kZQ);
        if (r < nrows) dst[r * kZXP + qq] = qok ? v[i] : cx<T>{T(0), T(0)};
    }
}

// Kz of one component, [j][kZQ] of this tile: each thread's elements
template <typename T>
struct KzShare {
    static constexpr int N = (kZJ * kZQ + kZThreads - 1) / kZThreads;
    cx<T> v[N];
    bool qok;
    __device__ __forceinline__ void load(const cx<T> *__restrict__ kzc, unsigned q0, int QP)
    {
        const unsigned qq = threadIdx.x % kZQ;
        qok = q0 + qq < (unsigned)QP;
        const cx<T> *base = kzc + (qok ? q0 + qq : 0u);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int j = (int)(threadIdx.x / kZQ) + i * (kZThreads / kZQ);
            v[i] = base[(size_t)(j < kZJ ? j : 0) * QP];
        }
    }
    __device__ __forceinline__ void put(cx<T> *ks) const
    {
        const unsigned qq = threadIdx.x % kZQ;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int j = (int)(threadIdx.x / kZQ) + i * (kZThreads / kZQ);
            if (j < kZJ) ks[j * kZKP + qq] = qok ? v[i] : cx<T>{T(0), T(0)};
        }
    }
};

// Kz of frequency j at this wave's position from the staged tile.
template <typename T>
__device__ __forceinline__ cx<T> kz_lds(const cx<T> *ks, unsigned j, unsigned qi)
{
    if (j < (unsigned)kZJ) return ks[j * kZKP + qi];
    return conjg(ks[(kZL - j) * kZKP + qi]);
}

// Plan time: Kz[row][c][j][q], j <= L/2, of the window of nwin spectral
// layers spec[m][row][c][q] (real).  One wave per (row, c, q); 16
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
        if (j < (unsigned)kZJ) kz[((size_t)rc * kZJ + j) * QP + q] = cx<TO>{(TO)v[s].re, (TO)v[s].im};
    }
}

// Forward: Dh[b][o - t0][c] for the chunk of levels o in [t0, t0 + tc), of
// every component of the group (Kz of the group: [U1][Cs][L/2+1][QP]); X is
// [B][nz][U1][2][QP], Dh [B][tc][Ct][U1][2][QP] (offset by the caller to the
// group's first slot).  The next component's Kz is loaded into registers
// while this one is transformed.
template <typename T>
__global__ void __launch_bounds__(kZThreads) __attribute__((amdgpu_waves_per_eu(4))) levelz_forward_kernel(const cx<T> *__restrict__ X,
                                                                  const cx<T> *__restrict__ kz, cx<T> *__restrict__ Dh,
                                                                  int nz, int t0, int tc, int U1, int QP, int Cs, int Ct,
                                                                  unsigned imag_mask, unsigned yodd_mask,
                                                                  const cx<T> *__restrict__ tw, int twlog)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ZTile z = ztile(QP);
    const unsigned b = blockIdx.y;
    const int nrows = nz > tc ? nz : tc;
    cx<T> *xs = reinterpret_cast<cx<T> *>(smem_raw);   // inputs, then outputs
    cx<T> *ks = xs + (size_t)nrows * kZXP;
    const size_t xslab = (size_t)U1 * 2 * QP;
    const cx<T> *kzr = kz + (size_t)z.row * Cs * kZJ * QP;
    KzShare<T> kn;
    kn.load(kzr, z.q0, QP);
    stage_tile(xs, X, (size_t)b * nz, 1, nz, xslab, z.row, z.h, z.q0, QP);
    __syncthreads();
    // conj of the transform of conj(X): sum_n X[n] W^{-j n}
    cx<T> y[4], t[9];
    if (z.active) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int n = (int)z.lane + 64 * s;
            y[s] = n < nz ? conjg(xs[n * kZXP + z.w]) : cx<T>{T(0), T(0)};
        }
        lane_twiddles<false>(t, tw, twlog, z.lane);
        lane_fft<false>(y, z.lane, t);
#pragma unroll
        for (int s = 0; s < 4; ++s) y[s] = conjg(y[s]);
        lane_twiddles<true>(t, tw, twlog, z.lane);
    }
    const T sc = T(1) / T(kZL);
    for (int c = 0; c < Cs; ++c) {
        kn.put(ks);
        __syncthreads();   // Kz of c staged; every wave is past its reads of the inputs or outputs
        if (c + 1 < Cs) kn.load(kzr + (size_t)(c + 1) * kZJ * QP, z.q0, QP);
        if (z.active) {
            cx<T> p[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) p[s] = mul(kz_lds(ks, zfreq<T>(z.lane, s), z.qi), y[s]);
            lane_fft<true>(p, z.lane, t);
            const bool im = (imag_mask >> c) & 1u, neg = z.h && ((yodd_mask >> c) & 1u);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int o = (int)z.lane + 64 * s;
                if (o >= t0 && o < t0 + tc) xs[(o - t0) * kZXP + z.w] = zfactor<T, false>(scale(p[s], sc), im, neg);
            }
        }
        __syncthreads();   // the outputs are staged; every wave is past its reads of Kz
        for (int e = (int)threadIdx.x; e < tc * kZQ; e += kZThreads) {
            const int r = e / kZQ, qq = e % kZQ;
            if (z.q0 + qq < (unsigned)QP)
                Dh[(((size_t)b * tc + r) * Ct + c) * xslab + ((size_t)z.row * 2 + z.h) * QP + z.q0 + qq] =
                    xs[r * kZXP + qq];
        }
    }
}

// Adjoint: Gh[b][n] (+)= sum_c sum_{t in chunk} K^_{c, n + t} Rh[b][t - t0][c]
// for n < nz; Rh is [B][tc][Ct][U1][2][QP] (offset to the group's first slot),
// Gh [B][nz][U1][2][QP].  Per component the inputs of the chunk are staged,
// transformed and multiplied by Kz into the sum; one inverse transform.
template <typename T>
__global__ void __launch_bounds__(kZThreads) __attribute__((amdgpu_waves_per_eu(4))) levelz_adjoint_kernel(const cx<T> *__restrict__ Rh,
                                                                  const cx<T> *__restrict__ kz, cx<T> *__restrict__ Gh,
                                                                  int nz, int t0, int tc, int U1, int QP, int Cs, int Ct,
                                                                  unsigned imag_mask, unsigned yodd_mask, int accumulate,
                                                                  const cx<T> *__restrict__ tw, int twlog)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ZTile z = ztile(QP);
    const unsigned b = blockIdx.y;
    const int nrows = nz > tc ? nz : tc;
    cx<T> *xs = reinterpret_cast<cx<T> *>(smem_raw);   // inputs of a component, then outputs
    cx<T> *ks = xs + (size_t)nrows * kZXP;
    const size_t xslab = (size_t)U1 * 2 * QP;
    const cx<T> *kzr = kz + (size_t)z.row * Cs * kZJ * QP;
    cx<T> t[9];
    lane_twiddles<false>(t, tw, twlog, z.lane);
    cx<T> acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = cx<T>{T(0), T(0)};
    for (int c = 0; c < Cs; ++c) {
        if (c > 0) __syncthreads();   // every wave is past its reads of the previous component
        {
            // Kz of c and the component's inputs (the other workgroup of the
            // CU transforms meanwhile)
            KzShare<T> kn;
            kn.load(kzr + (size_t)c * kZJ * QP, z.q0, QP);
            stage_tile(xs, Rh, (size_t)b * tc * Ct + c, (size_t)Ct, tc, xslab, z.row, z.h, z.q0, QP);
            kn.put(ks);
        }
        __syncthreads();
        if (z.active) {
            const bool im = (imag_mask >> c) & 1u, neg = z.h && ((yodd_mask >> c) & 1u);
            cx<T> y[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int tt = (int)z.lane + 64 * s;
                y[s] = (tt >= t0 && tt < t0 + tc) ? conjg(zfactor<T, true>(xs[(tt - t0) * kZXP + z.w], im, neg))
                                                  : cx<T>{T(0), T(0)};
            }
            lane_fft<false>(y, z.lane, t);
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[s] = add(acc[s], mul(kz_lds(ks, zfreq<T>(z.lane, s), z.qi), conjg(y[s])));
        }
    }
    __syncthreads();   // every wave is past its reads of the last inputs
    if (z.active) {
        lane_twiddles<true>(t, tw, twlog, z.lane);
        lane_fft<true>(acc, z.lane, t);
        const T sc = T(1) / T(kZL);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int n = (int)z.lane + 64 * s;
            if (n < nz) xs[n * kZXP + z.w] = scale(acc[s], sc);
        }
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < nz * kZQ; e += kZThreads) {
        const int r = e / kZQ, qq = e % kZQ;
        if (z.q0 + qq < (unsigned)QP) {
            cx<T> *dst = Gh + ((size_t)b * nz + r) * xslab + ((size_t)z.row * 2 + z.h) * QP + z.q0 + qq;
            cx<T> v = xs[r * kZXP + qq];
            if (accumulate) v = add(*dst, v);
            *dst = v;
        }
    }
}

}  // namespace

bool levelz_supported(int nwin) { return nwin >= 1 && nwin <= kZL; }

size_t levelz_values(int U1, int Cs, int QP) { return (size_t)U1 * Cs * kZJ * QP; }

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
    const dim3 grid((unsigned)(2 * U1 * ((QP + kZQ - 1) / kZQ)), (unsigned)B);
    const size_t lds = levelz_lds_bytes<double>(nz > tc ? nz : tc);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL(levelz_forward_kernel<double>, grid, dim3(kZThreads), lds, st, (const cx<double> *)X,
                       (const cx<double> *)kz, (cx<double> *)Dh, nz, t0, tc, U1, QP, Cs, Ct, imag_mask, yodd_mask,
                       (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_levelz_adjoint(const void *Rh, const void *kz, void *Gh, int B, int nz, int t0, int tc, int nt, int U1,
                          int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, bool accumulate,
                          const void *tw, int twlog, hipStream_t st)
{
    if (B < 1 || nz < 1 || tc < 1 || t0 < 0 || t0 + tc > nt || !levelz_supported(nz + nt - 1) || Cs < 1 ||
        Ct < Cs || twlog < 8)
        return -2;
    const dim3 grid((unsigned)(2 * U1 * ((QP + kZQ - 1) / kZQ)), (unsigned)B);
    const size_t lds = levelz_lds_bytes<double>(nz > tc ? nz : tc);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL(levelz_adjoint_kernel<double>, grid, dim3(kZThreads), lds, st, (const cx<double> *)Rh,
                       (const cx<double> *)kz, (cx<double> *)Gh, nz, t0, tc, U1, QP, Cs, Ct, imag_mask, yodd_mask,
                       accumulate ? 1 : 0, (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gf
