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
#include <type_traits>

#include "gf_fft.h"
#include "gf_lane.h"
#include "gf_launch.h"

namespace gf {

// Points per lane and radix of the column transforms.
template <typename T, int N>
struct ColShape {
    static constexpr int PPT = 8;
    static constexpr int RADIX = 8;
};

template <typename T, int N>
struct ColCfg {
    static constexpr int PPT = ColShape<T, N>::PPT;
    static constexpr int NT = N / PPT;
    static constexpr int RADIX = ColShape<T, N>::RADIX;
    // the transform of the hot passes: LDS twiddles
    using FFT = BlockFFT<T, N, NT, RADIX, false, true>;
    // the plan-time transform: full exchange, global twiddles
    using FFTK = BlockFFT<T, N, NT, RADIX, false, false>;
    static constexpr int W = FFT::lds_words();
    static constexpr int VEC = 16 / (int)sizeof(T);                  // values per 16 bytes
    static constexpr int up(int x) { return ((x + VEC - 1) / VEC) * VEC; }
    static constexpr int XW = up(2 * W);                              // exchange words (re, im)
    static constexpr int TWW = up(2 * FFT::stw_entries());            // per-stage twiddle table words
    static constexpr int QP = up(N / 2 + 1);                          // padded spectrum row
    static constexpr int CB = up(2 * (N / 2));                        // one column buffer (ldc <= N/2)
    // T words per group: exchange, twiddles and two spectrum buffers of cmax
    // rows (the density column of the next layer is prefetched into registers)
    static constexpr int group_words(int cmax, bool /*fwd*/) { return XW + TWW + 2 * cmax * QP; }
    // groups (column units) per workgroup: up to 256 threads for short
    // transforms, as long as the largest variant stays within 64 KB of LDS
    static constexpr int groups()
    {
        int g = NT >= 256 ? 1 : 256 / NT;
        while (g > 1 && (size_t)g * group_words(6, true) * sizeof(T) > 64 * 1024) g /= 2;
        return g;
    }
    static constexpr int G = groups();
    static constexpr int THREADS = G * NT;
    static constexpr bool ASYNC = (NT % 64) == 0;                     // groups are whole waves
    static constexpr size_t lds_bytes(int cmax, bool fwd) { return (size_t)G * group_words(cmax, fwd) * sizeof(T); }
    // register target: waves per SIMD of one workgroup (at least one) times
    // the workgroups per CU that fit in LDS (two in FP32, one in FP64)
    static constexpr int WAVES_PER_EU = (THREADS >= 256 ? THREADS / 256 : 1) * (sizeof(T) == 4 ? 2 : 1);
};

// Row of the resident spectra holding x-bin kx: rows are stored in the order
// kx = 0, Px/2, 1, 2, ..., Px/2-1 so that the two real-valued bins that share
// packed unit 0 are adjacent.
__device__ __forceinline__ unsigned spec_row(unsigned kx, unsigned M)
{
    return kx == 0 ? 0u : (kx == M ? 1u : kx + 1u);
}

// Copy `nvals` contiguous values (a multiple of 16 bytes) from global memory
// into this group's LDS buffer.  Whole-wave groups use the asynchronous
// global-to-LDS path (no registers; completion is awaited with a vmcnt wait);
// otherwise plain loads and stores.
template <typename T, int NT, bool ASYNC>
__device__ __forceinline__ void stage_rows(const T *__restrict__ src, T *dst, unsigned nvals, unsigned t)
{
    if constexpr (ASYNC) {
        constexpr unsigned VEC = 16 / sizeof(T);
        const unsigned nvec = nvals / VEC;
        const unsigned wave_off = __builtin_amdgcn_readfirstlane((t / 64) * 64);
        for (unsigned i = 0; i < nvec; i += NT) {
            if (i + t < nvec) {
                // lane l of the wave lands at LDS base + 16 l
                auto *lds = (__attribute__((address_space(3))) void *)(dst + (size_t)(i + wave_off) * VEC);
                __builtin_amdgcn_global_load_lds((const void *)(src + (size_t)(i + t) * VEC), lds, 16, 0, 0);
            }
        }
    } else {
        for (unsigned i = t; i < nvals; i += NT) dst[i] = src[i];
    }
}

// All of this wave's staged copies have landed, and every wave is past its
// reads of the buffers about to be refilled.
template <bool ASYNC>
__device__ __forceinline__ void stage_wait()
{
    if constexpr (ASYNC) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

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

// Column of unit u in a slab laid out [unit][y].  Units are the Px/2 x-bins
// kx = 1 .. Px/2-1 plus unit 0, which packs the two real-valued bins kx = 0
// (real part) and kx = Px/2 (imaginary part).
template <typename T>
__device__ __forceinline__ const cx<T> *column(const cx<T> *base, size_t slab, unsigned M, unsigned u,
                                               unsigned ny)
{
    return base + (slab * M + u) * (size_t)ny;
}

// Work of one group: virtual unit uv in [0, M] of model b.  uv = 0 and
// uv = M are the kx = 0 and kx = Px/2 bins, read from the real and the
// imaginary part of packed unit 0 and written back into them.
struct Unit {
    unsigned uv, u, b;
    int part;  // 0: whole complex column, 1: real part, 2: imaginary part
    bool active;
};

template <int NT, int G>
__device__ __forceinline__ Unit unit_of(unsigned g, int M, int B)
{
    Unit w;
    const unsigned U1 = (unsigned)M + 1;
    const unsigned gi = blockIdx.x * G + g;
    w.active = gi < U1 * (unsigned)B;
    w.uv = w.active ? gi / B : (unsigned)M;
    w.b = w.active ? gi % B : 0;
    if (NT >= 64) {  // a group is whole waves: keep its indices in scalar registers
        w.uv = __builtin_amdgcn_readfirstlane(w.uv);
        w.b = __builtin_amdgcn_readfirstlane(w.b);
    }
    w.u = (w.uv == (unsigned)M) ? 0u : w.uv;
    w.part = w.uv == 0 ? 1 : (w.uv == (unsigned)M ? 2 : 0);
    return w;
}

template <typename T>
__device__ __forceinline__ cx<T> take_part(cx<T> x, int part)
{
    if (part == 1) x.im = T(0);
    if (part == 2) x = cx<T>{x.im, T(0)};
    return x;
}

template <typename T, int PPT, typename F, int NT>
__device__ __forceinline__ void store_column(cx<T> *dst, const cx<T> (&v)[PPT], unsigned t, int ny, int part)
{
    T *dsc = reinterpret_cast<T *>(dst);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const unsigned y = t + NT * F::elem_out(s);
        if (y < (unsigned)ny) {
            if (part == 0)
                dst[y] = v[s];
            else
                dsc[2 * y + (part - 1)] = v[s].re;
        }
    }
}

// One component's term of the layer reduction, slot by slot:
// acc += K^ x (ADJ) or acc += conj(K^) x (forward), with K^ read from the
// quarter-plane row kr[ky], ky in [0, N/2].  K^ is k (real component) or i k
// (IM), and K^(N - ky) = -K^(ky) when the component is odd in y (YO).  A
// slot's half (ky below or above N/2) is fixed at compile time, so the
// mirrored index and the sign fold into addresses and operand modifiers;
// at ky = N/2 an odd component's spectrum is stored as exactly zero.
template <typename F, typename T, int PPT, int NT, int N, bool IM, bool YO, bool ADJ>
__device__ __forceinline__ void mac_component(cx<T> (&acc)[PPT], const cx<T> (&x)[PPT], const T *kr, unsigned t)
{
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const bool upper = F::elem_out(s) >= PPT / 2;
        const unsigned kq = upper ? (unsigned)(N - NT * F::elem_out(s)) - t : t + NT * F::elem_out(s);
        T k = kr[kq];
        if (YO && upper) k = -k;
        if (IM) {
            if (ADJ) {  // (i k) x
                acc[s].re -= k * x[s].im;
                acc[s].im += k * x[s].re;
            } else {    // conj(i k) x = -i k x
                acc[s].re += k * x[s].im;
                acc[s].im -= k * x[s].re;
            }
        } else {
            acc[s].re += k * x[s].re;
            acc[s].im += k * x[s].im;
        }
    }
}

template <typename F, typename T, int PPT, int NT, int N, bool ADJ>
__device__ __forceinline__ void mac_dispatch(cx<T> (&acc)[PPT], const cx<T> (&x)[PPT], const T *kr, unsigned t,
                                             bool im, bool yo)
{
    // im and yo are uniform across the workgroup: a scalar branch
    if (im) {
        if (yo) mac_component<F, T, PPT, NT, N, true, true, ADJ>(acc, x, kr, t);
        else    mac_component<F, T, PPT, NT, N, true, false, ADJ>(acc, x, kr, t);
    } else {
        if (yo) mac_component<F, T, PPT, NT, N, false, true, ADJ>(acc, x, kr, t);
        else    mac_component<F, T, PPT, NT, N, false, false, ADJ>(acc, x, kr, t);
    }
}

// Forward column pass.  Per layer n of the split: the density column of layer
// n+1 streams into registers and its spectrum rows into LDS (asynchronously)
// while layer n's column is transformed along y and each component
// accumulates conj(K^_{c,n}) times it; after the last layer one inverse
// transform per component.
template <typename T, int N, int CMAX, int KIND>
__global__ void __launch_bounds__((ColCfg<T, N>::THREADS))
    __attribute__((amdgpu_waves_per_eu(ColCfg<T, N>::WAVES_PER_EU)))
    col_forward_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec,
                       cx<T> *__restrict__ D, int B, int nz, int M, int ny, int ldc, int Cs, int Ct, int lps,
                       unsigned imag_mask, unsigned yodd_mask, const cx<T> *__restrict__ tw, int twlog)
{
    using C = ColCfg<T, N>;
    using F = typename C::FFT;
    // component kinds: compile-time for the common component sets (KIND >= 0:
    // bit c = imaginary spectrum, bit 8+c = odd in y), else the run-time masks
    const unsigned im_m = KIND >= 0 ? (unsigned)(KIND & 0xFF) : imag_mask;
    const unsigned yo_m = KIND >= 0 ? (unsigned)((KIND >> 8) & 0xFF) : yodd_mask;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, QP = C::QP;
    constexpr bool AS = C::ASYNC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    T *xbuf = lds + (size_t)g * C::group_words(CMAX, true);
    T *xim = xbuf + C::W;
    T *twq = xbuf + C::XW;
    T *sbuf = twq + C::TWW;                  // two spectrum buffers
    F::load_stage_table(twq, tw, twlog, t, NT);

    const Unit w = unit_of<NT, G>(g, M, B);
    const unsigned row = spec_row(w.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const int split = blockIdx.y;
    const int n0 = split * lps;
    const int n1 = min(nz, n0 + lps);
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);

    cx<T> acc[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
#pragma unroll
        for (int s = 0; s < PPT; ++s) acc[c][s] = cx<T>{T(0), T(0)};

    // the density column of the next layer travels into registers, its
    // spectrum rows into the other LDS buffer, while this layer is computed
    cx<T> vn[PPT] = {};
    auto load_col = [&](int n) {
        const cx<T> *col = column(R, (size_t)w.b * nz + n, M, w.u, ldc);
        // unconditional loads from a clamped row (a guarded load would wait
        // for its data at the branch join); rows past ny are zeroed on use.
        // Slots in the upper half (y >= N/2 >= ny) are the embedding's zero
        // padding and are never loaded.
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const unsigned y = t + NT * F::elem_in(s);
            if (F::elem_in(s) < PPT / 2) vn[s] = col[y < (unsigned)ny ? y : 0u];
        }
    };
    if (n0 < n1) {
        load_col(n0);
        stage_rows<T, NT, AS>(spec + (size_t)n0 * layer_vals + (size_t)row * Cs * QP, sbuf, (unsigned)Cs * QP, t);
    }
    stage_wait<AS>();

    for (int n = n0; n < n1; ++n) {
        const int cur = (n - n0) & 1;
        const T *scur = sbuf + cur * CMAX * QP;
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const unsigned y = t + NT * F::elem_in(s);
            v[s] = (F::elem_in(s) < PPT / 2 && y < (unsigned)ny) ? take_part(vn[s], w.part) : cx<T>{T(0), T(0)};
        }
        if (n + 1 < n1) {
            load_col(n + 1);
            stage_rows<T, NT, AS>(spec + (size_t)(n + 1) * layer_vals + (size_t)row * Cs * QP,
                                  sbuf + (cur ^ 1) * CMAX * QP, (unsigned)Cs * QP, t);
        }
        F::template run<false>(v, xbuf, xim, t, twp, twlog);
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < Cs)
                mac_dispatch<F, T, PPT, NT, N, false>(acc[c], v, scur + c * QP, t, (im_m >> c) & 1u,
                                                      (yo_m >> c) & 1u);
        stage_wait<AS>();
    }

#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        if (c < Cs) {
            out_to_in<F, T, PPT>(acc[c]);
            F::template run<true>(acc[c], xbuf, xim, t, twp, twlog);
            if (w.active)
                store_column<T, PPT, F, NT>(D + ((((size_t)split * B + w.b) * Ct + c) * M + w.u) * (size_t)ldc,
                                            acc[c], t, ny, w.part);
        }
    }
}

// Adjoint column pass: the Cs residual columns are transformed once; per
// layer the spectrum rows of the next layer stream into LDS while
// sum_c K^_{c,n} r^_c is formed and inverse-transformed.
template <typename T, int N, int CMAX, int KIND>
__global__ void __launch_bounds__((ColCfg<T, N>::THREADS))
    __attribute__((amdgpu_waves_per_eu(ColCfg<T, N>::WAVES_PER_EU)))
    col_adjoint_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec,
                       cx<T> *__restrict__ Gout, int B, int nz, int M, int ny, int ldc, int Cs, int Ct, int lps,
                       unsigned imag_mask, unsigned yodd_mask, const cx<T> *__restrict__ tw, int twlog)
{
    using C = ColCfg<T, N>;
    using F = typename C::FFT;
    // component kinds: compile-time for the common component sets (KIND >= 0:
    // bit c = imaginary spectrum, bit 8+c = odd in y), else the run-time masks
    const unsigned im_m = KIND >= 0 ? (unsigned)(KIND & 0xFF) : imag_mask;
    const unsigned yo_m = KIND >= 0 ? (unsigned)((KIND >> 8) & 0xFF) : yodd_mask;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, QP = C::QP;
    constexpr bool AS = C::ASYNC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    T *xbuf = lds + (size_t)g * C::group_words(CMAX, false);
    T *xim = xbuf + C::W;
    T *twq = xbuf + C::XW;
    T *sbuf = twq + C::TWW;
    F::load_stage_table(twq, tw, twlog, t, NT);
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);

    const Unit w = unit_of<NT, G>(g, M, B);
    const unsigned row = spec_row(w.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const int split = blockIdx.y;
    const int n0 = split * lps;
    const int n1 = min(nz, n0 + lps);

    cx<T> rh[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
#pragma unroll
        for (int s = 0; s < PPT; ++s) rh[c][s] = cx<T>{T(0), T(0)};
        if (c < Cs) {  // unconditional loads from clamped rows, selected after
            const cx<T> *col = column(R, (size_t)w.b * Ct + c, M, w.u, ldc);
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const unsigned y = t + NT * F::elem_in(s);
                if (F::elem_in(s) < PPT / 2) rh[c][s] = col[y < (unsigned)ny ? y : 0u];   // upper half: padding
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const unsigned y = t + NT * F::elem_in(s);
            rh[c][s] = (F::elem_in(s) < PPT / 2 && y < (unsigned)ny) ? take_part(rh[c][s], w.part)
                                                                       : cx<T>{T(0), T(0)};
        }
    __syncthreads();   // twiddle table complete
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
        if (c < Cs) F::template run<false>(rh[c], xbuf, xim, t, twp, twlog);

    if (n0 < n1)
        stage_rows<T, NT, AS>(spec + (size_t)n0 * layer_vals + (size_t)row * Cs * QP, sbuf, (unsigned)Cs * QP, t);
    stage_wait<AS>();

    for (int n = n0; n < n1; ++n) {
        const int cur = (n - n0) & 1;
        const T *scur = sbuf + cur * CMAX * QP;
        if (n + 1 < n1)
            stage_rows<T, NT, AS>(spec + (size_t)(n + 1) * layer_vals + (size_t)row * Cs * QP,
                                  sbuf + (cur ^ 1) * CMAX * QP, (unsigned)Cs * QP, t);
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) v[s] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < Cs)
                mac_dispatch<F, T, PPT, NT, N, true>(v, rh[c], scur + c * QP, t, (im_m >> c) & 1u,
                                                     (yo_m >> c) & 1u);
        out_to_in<F, T, PPT>(v);
        F::template run<true>(v, xbuf, xim, t, twp, twlog);
        if (w.active)
            store_column<T, PPT, F, NT>(Gout + (((size_t)w.b * nz + n) * M + w.u) * (size_t)ldc, v, t, ny, w.part);
        stage_wait<AS>();
    }
}

// ---------------------------------------------------------------------------
// Wave-split column passes (transform lengths N >= 512).
//
// One decimation-in-frequency step splits a length-N column transform into
// NW = N / L independent transforms of length L = 64 * PPT, one per wave:
//     X[NW k2 + w] = sum_{n2 < L} W_L^{n2 k2} z_w[n2],
//     z_w[n2] = W_N^{n2 w} sum_{n1 < NW} W_NW^{n1 w} x[n2 + L n1],
// where only n1 < NW/2 contribute (rows y >= N/2 are the zero padding of the
// circulant embedding).  Wave w forms z_w from the column (staged in LDS),
// transforms it with wave-local exchanges (no workgroup barrier) and owns the
// frequencies ky = NW k2 + w in the layer reduction.  The inverse transform
// runs the same split backwards: wave w inverse-transforms its frequencies to
// Y_w[m'], m' < L, and the output is
//     y[m' + L j] = sum_w W_NW^{-j w} W_N^{-m' w} Y_w[m'],
// a combination of the waves through LDS once per output column.
//
// Resident spectrum rows are stored in residue-block order (spec_pos), so
// that the frequencies of one wave are contiguous in LDS.
#ifndef GF_WS_PPT64
#define GF_WS_PPT64 4
#endif
#ifndef GF_WS_PPT32
#define GF_WS_PPT32 8
#endif
// Points per lane of the wave transforms for column length N: four in FP64
// (two waves per SIMD fit the accumulators); in FP32 four up to length 1024
// (in-register transforms; the batched 512 x 512 x 128 adjoint column pass
// 6.25 -> 4.75 ms against eight) and eight beyond (fewer column reads
// through LDS: the 2048-point forward 0.69 -> 0.68 ms against four),
// adjusted so that a column has one to eight waves.  The spectrum layout
// follows it, so it is fixed per plan precision and column length.
template <typename T, int N>
constexpr int ws_ppt()
{
    int p = sizeof(T) == 8 ? GF_WS_PPT64 : (N <= 1024 ? 4 : GF_WS_PPT32);
    while (p > 1 && 64 * p > N) p /= 2;
    while (N / (64 * p) > 8) p *= 2;
    return p;
}

// Transform lengths that run in the wave split.
template <int N>
constexpr bool use_ws() { return N >= 256; }

// Waves per column of the wave split (1 for lengths that do not use it).
template <typename T, int N>
constexpr int ws_waves() { return use_ws<N>() ? N / (64 * ws_ppt<T, N>()) : 1; }

// The wave transform of the wave split: in registers for four points a lane,
// else the LDS-exchange block transform (xch, twp: its exchange array and
// stage table; ltw: the in-register transform's lane twiddles).
template <bool INV, typename F, typename T, int PPT>
__device__ __forceinline__ void ws_fft(cx<T> (&v)[PPT], T *xch, unsigned lane, const cx<T> *twp, int twlog,
                                       const cx<T> *ltw)
{
    if constexpr (is_lane_fft<F>::value) lane_fft<INV>(v, lane, ltw);
    else F::template run<INV>(v, xch, nullptr, lane, twp, twlog);
}

#ifndef GF_WS_SH_WAVES
#define GF_WS_SH_WAVES 3
#endif
// Layout and launch shape of the wave-split passes.  Unshared (SH false):
// each column group of a workgroup owns one (column unit, model) item with
// its own spectrum buffers.  Shared (SH): the groups of a workgroup (256
// threads, or 512 for columns of four or more waves) are models of one
// column unit, staging its spectrum rows once into one set of buffers, which
// leaves LDS for more resident waves when a batch of models shares the
// geometry (up to GF_WS_SH_WAVES a SIMD: the accumulators of six spectra
// take most of the registers of three).
template <typename T, int N, bool SH = false>
struct WsCfg {
    static constexpr int PPT = ws_ppt<T, N>();
    static constexpr int L = 64 * PPT;                                // one wave's transform length
    static constexpr int NW = N / L;                                  // waves per column
    static constexpr int GT = 64 * NW;                                // threads per column
    static constexpr int G = SH ? (GT <= 128 ? 256 / GT : (GT >= 512 ? 1 : 512 / GT))
                                : (NW >= 4 ? 1 : 4 / NW);             // columns per workgroup
    static constexpr int THREADS = G * GT;
    // four points a lane: the in-register transform; eight: LDS exchanges
    static constexpr bool LANE = PPT == 4;
    using FFT = typename std::conditional<LANE, LaneFFT<T>, BlockFFT<T, L, 64, (PPT >= 8 ? 8 : PPT), true, true, true>>::type;
    static constexpr int VEC = 16 / (int)sizeof(T);
    static constexpr int up(int x) { return ((x + VEC - 1) / VEC) * VEC; }
    static constexpr int XW = up(FFT::lds_words());                   // one wave's exchange array
    static constexpr int TWW = up(2 * FFT::stw_entries());            // stage twiddles, shared
    static constexpr int QP = up(N / 2 + 1);                          // padded spectrum row
    static constexpr int CW = N;                                      // one column buffer (N/2 complex)
    static constexpr int GW = 2 * CW + NW * XW;                       // a group's columns and exchange arrays
    // T words per column: nbuf spectrum buffers, two column buffers and the
    // waves' exchange arrays (the spectrum buffers once per workgroup when
    // shared).  At the end, 2N words of the group (re, im of N values) hold
    // the combination of the waves' inverse transforms: the start of its
    // area (unshared) or its column buffers (shared).
    static constexpr int words_with(int nbuf, int cmax) { return nbuf * cmax * QP + GW; }
    static constexpr size_t bytes_with(int nbuf, int cmax)
    {
        return SH ? ((size_t)nbuf * cmax * QP + (size_t)G * GW + TWW) * sizeof(T)
                  : ((size_t)G * words_with(nbuf, cmax) + TWW) * sizeof(T);
    }
    static constexpr int fit(size_t bytes) { return (int)(163840 / bytes); }
    // Two spectrum buffers (the next layer's rows stream in while this layer
    // is reduced) unless only one fits in the 160 KB of LDS of a CU (FP64 at
    // length 4096 holds three spectra with one buffer, one with two), or,
    // shared, unless one buffer fits more workgroups per CU (up to two).  With
    // one buffer the next layer's rows stream in while the next column is
    // transformed.
    static constexpr int WPW = THREADS >= 256 ? THREADS / 256 : 1;   // waves per SIMD of one workgroup
    static constexpr int WG_CAP = SH ? (GF_WS_SH_WAVES / WPW > 0 ? GF_WS_SH_WAVES / WPW : 1) : 64;
    static constexpr int fit_capped(size_t bytes) { return fit(bytes) < WG_CAP ? fit(bytes) : WG_CAP; }
    static constexpr bool single_spec(int cmax)
    {
        if (SH) return fit_capped(bytes_with(2, cmax)) < fit_capped(bytes_with(1, cmax));
        return bytes_with(2, cmax) > 163840 && bytes_with(1, cmax) <= 163840;
    }
    static constexpr int spec_bufs(int cmax) { return single_spec(cmax) ? 1 : 2; }
    static constexpr int group_words(int cmax) { return SH ? GW : words_with(spec_bufs(cmax), cmax); }
    static constexpr size_t lds_bytes(int cmax) { return bytes_with(spec_bufs(cmax), cmax); }
    // register target: waves per SIMD of the workgroups that fit in 160 KB of
    // LDS (shared: capped as above)
    static constexpr int WG_PER_CU = fit_capped(lds_bytes(6)) > 0 ? fit_capped(lds_bytes(6)) : 1;
    static constexpr int WAVES_PER_EU = WPW * WG_PER_CU;
    static_assert(N % L == 0 && NW >= 1 && NW <= 8, "wave split needs N = NW * L with NW in 1..8");
};

// Whether the shared layout serves a batch of B models at length N: it
// exists where a workgroup holds two or more columns, and runs when the
// models fill its groups (few idle groups).
template <typename T, int N>
constexpr bool ws_shared_exists()
{
    if constexpr (use_ws<N>())
        return WsCfg<T, N, true>::G >= 2 && WsCfg<T, N, true>::WAVES_PER_EU > WsCfg<T, N, false>::WAVES_PER_EU;
    else
        return false;
}
template <typename T, int N>
inline bool ws_shared_for(int B)
{
    constexpr int G = WsCfg<T, N, true>::G;
    return ws_shared_exists<T, N>() && B >= 2 && (B % G == 0 || B >= 2 * G);
}

// Whether resident rows at column length N are stored in the lane order of
// the in-register wave transform (see spec_pos).
template <typename T, int N>
constexpr bool ws_lane_order() { return use_ws<N>() && ws_ppt<T, N>() == 4; }

// Base-4 digit reversal of a 6-bit index (an involution): the lane of the
// in-register transform's output that holds frequency index x mod 64.
__host__ __device__ constexpr unsigned digit_rev64(unsigned x)
{
    return (x >> 4) + 4u * ((x >> 2) & 3u) + 16u * (x & 3u);
}

// Position of frequency ky in [0, N/2] within a resident spectrum row:
// residue blocks r = ky mod NW (block 0 holds N/(2 NW) + 1 values, the
// others N/(2 NW)), index j = ky / NW within a block.  Where the wave
// transform runs in registers its output frequencies sit in lanes in
// digit-reversed order, so each 64-value chunk of a block is stored in that
// order: lane l then reads the l-th value of a chunk (its own frequencies)
// or the (63 - l)-th (the mirrored ones), and the reads of a wave meet
// distinct LDS banks.
template <typename T, int N>
__host__ __device__ constexpr unsigned spec_pos(unsigned ky)
{
    constexpr unsigned NW = (unsigned)ws_waves<T, N>();
    const unsigned r = NW == 1 ? 0u : ky % NW, j = NW == 1 ? ky : ky / NW;
    const unsigned base = r == 0 ? 0u : r * (N / NW / 2) + 1u;
    if (ws_lane_order<T, N>() && j < (unsigned)(N / NW / 2)) return base + (j & ~63u) + digit_rev64(j & 63u);
    return base + j;
}

// exp(-2 pi i k / n) * x for a compile-time k and n in {1, 2, 4, 8}
template <typename T, int K, int NN>
__device__ __forceinline__ cx<T> wpow(cx<T> x)
{
    constexpr int k8 = ((K % NN + NN) % NN) * (8 / NN);   // in eighths of a turn
    const T h = T(0.70710678118654752440084436210484903928);
    if constexpr (k8 == 0) return x;
    else if constexpr (k8 == 1) return cx<T>{(x.re + x.im) * h, (x.im - x.re) * h};
    else if constexpr (k8 == 2) return cx<T>{x.im, -x.re};
    else if constexpr (k8 == 3) return cx<T>{(x.im - x.re) * h, -(x.re + x.im) * h};
    else if constexpr (k8 == 4) return cx<T>{-x.re, -x.im};
    else if constexpr (k8 == 5) return cx<T>{-(x.re + x.im) * h, (x.re - x.im) * h};
    else if constexpr (k8 == 6) return cx<T>{-x.im, x.re};
    else return cx<T>{(x.re - x.im) * h, (x.re + x.im) * h};
}

// Stage `nvals` (a multiple of 16 bytes) plus, for an odd number of FP32
// complex values, the last value through a register: the column copy of a
// group.  `tail` carries that value until it is written to LDS.
template <typename T, int GT>
__device__ __forceinline__ void stage_column(const cx<T> *__restrict__ col, cx<T> *dst, int ny, unsigned tg,
                                             cx<T> &tail)
{
    constexpr int PER = 16 / (int)sizeof(cx<T>);   // complex values per 16 bytes
    const int nfull = (ny / PER) * PER;
    stage_rows<T, GT, true>(reinterpret_cast<const T *>(col), reinterpret_cast<T *>(dst), 2u * (unsigned)nfull, tg);
    if (PER > 1 && nfull < ny && tg == 0) tail = col[ny - 1];
}

template <typename T>
__device__ __forceinline__ void put_tail(cx<T> *dst, int ny, unsigned tg, const cx<T> &tail)
{
    constexpr int PER = 16 / (int)sizeof(cx<T>);
    if (PER > 1 && (ny % PER) != 0 && tg == 0) dst[ny - 1] = tail;
}

// Twiddles of the wave split: W_N^{(lane + 64 e) w} = base * cw[e].
template <typename T, int N, int PPT>
struct WsTwiddles {
    cx<T> base;
    cx<T> cw[PPT];
    __device__ __forceinline__ void init(const cx<T> *__restrict__ tw, int twlog, unsigned lane, unsigned w)
    {
        constexpr int LOGN = ilog2<N>::value;
        const unsigned sh = (unsigned)(twlog - LOGN);
        base = tw[((lane * w) & (N - 1)) << sh];
#pragma unroll
        for (int e = 0; e < PPT; ++e) cw[e] = tw[((64u * e * w) & (N - 1)) << sh];
    }
    template <bool INV>
    __device__ __forceinline__ cx<T> apply(cx<T> x, int e) const
    {
        const cx<T> t = mul(base, cw[e]);
        return mul(x, INV ? conjg(t) : t);
    }
};

// z_w of the wave split for this lane's slots (FFT input layout), from the
// column staged in LDS (xc: N/2 values, zero beyond the data; every index
// read is below N/2: n2 + L n1 < L NW/2 for NW > 1, and with one wave the
// slots at n2 >= N/2 are the padding).  PART selects the real (1) or
// imaginary (2) part of a packed column, 0 the whole value.
template <typename F, typename T, int N, int NW, int L, int PPT, int PART>
__device__ __forceinline__ void form_z(cx<T> (&v)[PPT], const cx<T> *xc, unsigned lane, unsigned w,
                                       const cx<T> (&cn)[NW > 1 ? NW / 2 : 1], const WsTwiddles<T, N, PPT> &tws)
{
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const unsigned n2 = lane + 64u * F::elem_in(s);
        if (NW == 1 && F::elem_in(s) >= PPT / 2) {   // n2 >= N/2: zero padding, not staged
            v[s] = cx<T>{T(0), T(0)};
            continue;
        }
        cx<T> a = take_part(xc[n2], PART);
#pragma unroll
        for (int n1 = 1; n1 < NW / 2; ++n1) {
            const cx<T> b = take_part(xc[n2 + (unsigned)L * n1], PART);
            a = add(a, mul(cn[n1], b));
        }
        v[s] = NW > 1 ? tws.template apply<false>(a, F::elem_in(s)) : a;
    }
}

// Offsets of wave w's frequencies in a residue-ordered spectrum row (slot
// s of a lane holds k2 = ws_out_lane(lane) + 64 e after the forward
// transform): lower slots (ky = NW k2 + w <= N/2, block w, index k2) and
// upper slots (their mirror N - ky: block NW - w, index L - 1 - k2, or block
// 0, index L - k2, for w = 0), at the positions spec_pos gives them.  In the
// lane order that is lo + lane + 64 e and hi - lane - 64 e, except for the
// upper slots of wave 0, whose mirrored indices L - k2 are one off the
// chunk boundaries.
template <typename F, int PPT, int NW, int L>
__device__ __forceinline__ void ws_spec_offsets(unsigned (&off)[PPT], unsigned lane, unsigned w)
{
    const unsigned lo = w == 0 ? 0u : w * (L / 2) + 1u;
    const unsigned hi = w == 0 ? (unsigned)L : (NW - w) * (L / 2) + (unsigned)L;
    const unsigned ol = ws_out_lane<F>(lane);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const unsigned e = (unsigned)F::elem_out(s);
        const bool upper = F::elem_out(s) >= PPT / 2;
        if constexpr (is_lane_fft<F>::value) {
            static_assert(L == 256, "the lane order holds for the 256-point in-register transform");
            if (!upper) {
                off[s] = lo + lane + 64u * e;
            } else if (w != 0) {
                off[s] = hi - lane - 64u * e;
            } else {
                const unsigned j = (unsigned)L - ol - 64u * e;
                off[s] = j < (unsigned)(L / 2) ? (j & ~63u) + digit_rev64(j & 63u) : j;
            }
        } else {
            const unsigned k2 = ol + 64u * e;
            off[s] = upper ? hi - k2 : lo + k2;
        }
    }
}

// One component's term of the layer reduction in the wave split (see
// mac_component for the kinds): slot s of this lane reads its spectrum value
// at kr[off[s]].
template <typename F, typename T, int PPT, int NW, bool IM, bool YO, bool ADJ>
__device__ __forceinline__ void mac_ws(cx<T> (&acc)[PPT], const cx<T> (&x)[PPT], const T *kr,
                                       const unsigned (&off)[PPT])
{
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const bool upper = F::elem_out(s) >= PPT / 2;
        T k = kr[off[s]];
        if (YO && upper) k = -k;
        if (IM) {
            if (ADJ) {
                acc[s].re -= k * x[s].im;
                acc[s].im += k * x[s].re;
            } else {
                acc[s].re += k * x[s].im;
                acc[s].im -= k * x[s].re;
            }
        } else {
            acc[s].re += k * x[s].re;
            acc[s].im += k * x[s].im;
        }
    }
}

template <typename F, typename T, int PPT, int NW, bool ADJ>
__device__ __forceinline__ void mac_ws_dispatch(cx<T> (&acc)[PPT], const cx<T> (&x)[PPT], const T *kr,
                                                const unsigned (&off)[PPT], bool im, bool yo)
{
    if (im) {
        if (yo) mac_ws<F, T, PPT, NW, true, true, ADJ>(acc, x, kr, off);
        else    mac_ws<F, T, PPT, NW, true, false, ADJ>(acc, x, kr, off);
    } else {
        if (yo) mac_ws<F, T, PPT, NW, false, true, ADJ>(acc, x, kr, off);
        else    mac_ws<F, T, PPT, NW, false, false, ADJ>(acc, x, kr, off);
    }
}

// Inverse transform of this wave's frequencies (v in FFT output layout) and
// its contribution W_N^{-m' w} Y_w[m'] written to the combination arrays
// (re at cre[w L + m'], im at cre[N + w L + m']).
template <typename F, typename T, int N, int NW, int L, int PPT>
__device__ __forceinline__ void ws_inverse_put(cx<T> (&v)[PPT], T *xch, const cx<T> *twp, int twlog, unsigned lane,
                                               unsigned w, const WsTwiddles<T, N, PPT> &tws, T *cre, const cx<T> *ltw)
{
    // the in-register transform takes the forward's output layout as it is
    if constexpr (!is_lane_fft<F>::value) out_to_in<F, T, PPT>(v);
    ws_fft<true, F>(v, xch, lane, twp, twlog, ltw);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const unsigned m = lane + 64u * F::elem_out(s);
        const cx<T> a = NW > 1 ? tws.template apply<true>(v[s], F::elem_out(s)) : v[s];
        cre[w * L + m] = a.re;
        cre[N + w * L + m] = a.im;
    }
}

// Output value m' + L j of the combination (after a barrier), j compile-time.
template <typename T, int N, int NW, int L, int J, int WI = 0>
__device__ __forceinline__ cx<T> ws_combine(const T *cre, unsigned mp)
{
    if constexpr (WI == NW) {
        return cx<T>{T(0), T(0)};
    } else {
        const cx<T> a{cre[WI * L + mp], cre[N + WI * L + mp]};
        return add(wpow<T, -J * WI, NW>(a), ws_combine<T, N, NW, L, J, WI + 1>(cre, mp));
    }
}

// ws_combine for a block index j in [JJ, NW/2) known only at run time (it is
// uniform across a wave: blocks of L rows are whole waves of rows).
template <typename T, int N, int NW, int L, int JJ = 0>
__device__ __forceinline__ cx<T> ws_combine_j(const T *cre, unsigned mp, unsigned j)
{
    if constexpr (JJ + 1 >= NW / 2 || NW == 1) {
        return ws_combine<T, N, NW, L, JJ>(cre, mp);
    } else {
        if (j == (unsigned)JJ) return ws_combine<T, N, NW, L, JJ>(cre, mp);
        return ws_combine_j<T, N, NW, L, JJ + 1>(cre, mp, j);
    }
}

// Outputs y < ny of the combined column: thread tg of the group writes
// y = tg + GT q, q < (N/2)/GT (consecutive threads, consecutive rows).
// part: 0 complex column, 1 / 2 the real / imaginary field of a packed
// column, 3 a real column (array of T).
// ws_combine from the NW values of one m' already in registers (the same
// sum, in the same order).
template <typename T, int NW, int J, int WI = 0>
__device__ __forceinline__ cx<T> ws_combine_regs(const cx<T> (&a)[NW])
{
    if constexpr (WI == NW) {
        return cx<T>{T(0), T(0)};
    } else {
        return add(wpow<T, -J * WI, NW>(a[WI]), ws_combine_regs<T, NW, J, WI + 1>(a));
    }
}

template <typename T, int NW, int JJ = 0>
__device__ __forceinline__ cx<T> ws_combine_regs_j(const cx<T> (&a)[NW], unsigned j)
{
    if constexpr (JJ + 1 >= NW / 2) {
        return ws_combine_regs<T, NW, JJ>(a);
    } else {
        if (j == (unsigned)JJ) return ws_combine_regs<T, NW, JJ>(a);
        return ws_combine_regs_j<T, NW, JJ + 1>(a, j);
    }
}

template <typename T>
__device__ __forceinline__ void ws_put(cx<T> *dst, unsigned y, const cx<T> &r, int part)
{
    if (part == 0)
        dst[y] = r;
    else if (part == 3)
        reinterpret_cast<T *>(dst)[y] = r.re;
    else
        reinterpret_cast<T *>(dst)[2 * y + (part - 1)] = r.re;
}

template <typename T, int N, int NW, int L, int PPT, int GT, int Q = 0>
__device__ __forceinline__ void ws_store(const T *cre, cx<T> *dst, unsigned tg, int ny, int part)
{
    if constexpr (Q == 0 && NW > 1 && GT % L == 0 && (N / 2) / GT > 1) {
        // every output row of this thread has the same m' = tg mod L (rows
        // GT apart, GT a multiple of L): read the NW wave values once
        const unsigned mp = tg % (unsigned)L, j0 = tg / (unsigned)L;
        cx<T> a[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) a[w] = cx<T>{cre[w * L + mp], cre[N + w * L + mp]};
#pragma unroll
        for (int q = 0; q < (N / 2) / GT; ++q) {
            const unsigned y = tg + (unsigned)(GT * q);
            if (y < (unsigned)ny) ws_put(dst, y, ws_combine_regs_j<T, NW>(a, j0 + (unsigned)(q * (GT / L))), part);
        }
    } else if constexpr (Q < (N / 2) / GT) {
        const unsigned y = tg + (unsigned)(GT * Q);
        if (y < (unsigned)ny) {
            const unsigned j = y / (unsigned)L;
            const cx<T> r = ws_combine_j<T, N, NW, L>(cre, y - (unsigned)L * j, j);
            if (part == 0)
                dst[y] = r;
            else if (part == 3)
                reinterpret_cast<T *>(dst)[y] = r.re;
            else
                reinterpret_cast<T *>(dst)[2 * y + (part - 1)] = r.re;
        }
        ws_store<T, N, NW, L, PPT, GT, Q + 1>(cre, dst, tg, ny, part);
    }
}

// Work of one group in the wave-split passes.  The grid is one-dimensional:
// blocks [0, nblk_ny) hold the chunks of the real Nyquist unit (kx = Px/2,
// the imaginary part of packed unit 0), Sny chunks of lps_ny layers per
// model (nblk_ny = Sny * ceil(B / G)); the other blocks hold the Px/2 main
// units (uv = 0, the real kx = 0 column, and the complex bins 1 .. Px/2-1)
// of every model, split by layers into S splits of lps layers (nblk_main
// blocks per split).  Keeping the odd Nyquist unit out of the main grid lets
// the main grid fill whole rounds of the device.  All groups of a block run
// the same layers.
struct WsItem {
    unsigned uv, u, b;
    int part;        // 0: complex column, 1: real part of unit 0, 2: imaginary part of unit 0
    int n0, n1;      // layers
    int split;       // split index (main) or chunk index (Nyquist)
    bool active, nyq;
};

template <int GT, int G, bool SH = false>
__device__ __forceinline__ WsItem ws_item(unsigned g, int M, int B, int nz, int lps, int nblk_ny, int Sny,
                                          int lps_ny, int nblk_main)
{
    WsItem it;
    const unsigned bx = blockIdx.x;
    if ((int)bx < nblk_ny) {
        // every group of a block takes the same chunk (the layer loop holds
        // workgroup barriers, so its trip count must be uniform), models
        // across the groups
        const unsigned nbb = ((unsigned)B + G - 1) / G;
        const unsigned bb = (bx % nbb) * G + g;
        it.active = bb < (unsigned)B;
        it.b = it.active ? bb : 0u;
        it.split = (int)(bx / nbb);
        it.uv = (unsigned)M;
        it.u = 0;
        it.part = 2;
        it.nyq = true;
        it.n0 = it.split * lps_ny;
        it.n1 = min(nz, it.n0 + lps_ny);
    } else {
        const unsigned bm = bx - (unsigned)nblk_ny;
        it.split = (int)(bm / (unsigned)nblk_main);
        if constexpr (SH) {
            // the groups are models of one unit: nblk_main = M * ceil(B / G)
            const unsigned nbb = ((unsigned)B + G - 1) / G, r = bm % (unsigned)nblk_main;
            const unsigned bb = (r % nbb) * G + g;
            it.active = bb < (unsigned)B;
            it.uv = r / nbb;
            it.b = it.active ? bb : 0u;
        } else {
            const unsigned gi = (bm % (unsigned)nblk_main) * G + g;
            it.active = gi < (unsigned)M * (unsigned)B;
            const unsigned gc = it.active ? gi : 0u;
            it.uv = gc / (unsigned)B;
            it.b = gc % (unsigned)B;
        }
        it.u = it.uv;
        it.part = it.uv == 0 ? 1 : 0;
        it.nyq = false;
        it.n0 = it.split * lps;
        it.n1 = min(nz, it.n0 + lps);
    }
    it.uv = __builtin_amdgcn_readfirstlane(it.uv);
    it.u = __builtin_amdgcn_readfirstlane(it.u);
    it.b = __builtin_amdgcn_readfirstlane(it.b);
    it.n0 = __builtin_amdgcn_readfirstlane(it.n0);
    it.n1 = __builtin_amdgcn_readfirstlane(it.n1);
    return it;
}

template <typename T, int N, int CMAX, int KIND, bool SH>
__global__ void __launch_bounds__((WsCfg<T, N, SH>::THREADS))
    __attribute__((amdgpu_waves_per_eu(WsCfg<T, N, SH>::WAVES_PER_EU)))
    col_forward_ws_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec, cx<T> *__restrict__ D,
                          T *__restrict__ Dny, int B, int nz, int M, int ny, int ldc, int Cs, int Ct, int lps,
                          int nblk_ny, int Sny, int lps_ny, int nblk_main, unsigned imag_mask,
                          unsigned yodd_mask, const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N, SH>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    const unsigned im_m = KIND >= 0 ? (unsigned)(KIND & 0xFF) : imag_mask;
    const unsigned yo_m = KIND >= 0 ? (unsigned)((KIND >> 8) & 0xFF) : yodd_mask;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    constexpr int NB = C::spec_bufs(CMAX);
    // spectrum rows are staged by the group (unshared) or by the workgroup (shared)
    constexpr int ST = SH ? C::THREADS : GT;
    const unsigned ts = SH ? threadIdx.x : tg;
    T *twq = lds;
    T *gb = lds + C::TWW + (SH ? NB * CMAX * QP : 0) + (size_t)g * C::group_words(CMAX);
    T *sbuf = SH ? lds + C::TWW : gb;                                    // NB x CMAX x QP
    T *cw = SH ? gb : gb + NB * CMAX * QP;
    cx<T> *cbuf = reinterpret_cast<cx<T> *>(cw);                         // 2 x N/2 complex
    T *xch = cw + 2 * C::CW + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);
    for (unsigned i = (unsigned)ny + tg; i < (unsigned)(N / 2); i += GT) {
        cbuf[i] = cx<T>{T(0), T(0)};
        cbuf[N / 2 + i] = cx<T>{T(0), T(0)};
    }

    WsTwiddles<T, N, PPT> tws;
    cx<T> cn[NW > 1 ? NW / 2 : 1];
    if constexpr (NW > 1) {
        tws.init(tw, twlog, lane, w);
        constexpr int LOGN = ilog2<N>::value;
#pragma unroll
        for (int n1 = 0; n1 < NW / 2; ++n1) cn[n1] = tw[(((unsigned)L * n1 * w) & (N - 1)) << (twlog - LOGN)];
    }
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<false>(ltw, tw, twlog, lane);

    const WsItem un = ws_item<GT, G, SH>(g, M, B, nz, lps, nblk_ny, Sny, lps_ny, nblk_main);
    const unsigned row = spec_row(un.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const int n0 = un.n0;
    const int n1 = un.n1;

    cx<T> acc[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
#pragma unroll
        for (int s = 0; s < PPT; ++s) acc[c][s] = cx<T>{T(0), T(0)};

    cx<T> tail{T(0), T(0)};
    auto stage_spec = [&](int n, int buf) {
        stage_rows<T, ST, true>(spec + (size_t)n * layer_vals + (size_t)row * Cs * QP, sbuf + buf * CMAX * QP,
                                (unsigned)Cs * QP, ts);
    };
    auto stage_col = [&](int n, int buf) {
        stage_column<T, GT>(column(R, (size_t)un.b * nz + n, M, un.u, ldc), cbuf + buf * (N / 2), ny, tg, tail);
    };
    if (n0 < n1) {
        stage_spec(n0, 0);
        stage_col(n0, 0);
        put_tail(cbuf, ny, tg, tail);
    }
    stage_wait<true>();

    for (int n = n0; n < n1; ++n) {
        const int cur = (n - n0) & 1;
        if (n + 1 < n1) {
            if constexpr (NB == 2) stage_spec(n + 1, cur ^ 1);
            stage_col(n + 1, cur ^ 1);
        }
        cx<T> v[PPT];
        const cx<T> *xc = cbuf + cur * (N / 2);
        if (un.part == 0)
            form_z<F, T, N, NW, L, PPT, 0>(v, xc, lane, w, cn, tws);
        else if (un.part == 1)
            form_z<F, T, N, NW, L, PPT, 1>(v, xc, lane, w, cn, tws);
        else
            form_z<F, T, N, NW, L, PPT, 2>(v, xc, lane, w, cn, tws);
        ws_fft<false, F>(v, xch, lane, twp, twlog, ltw);
        // one buffer: this layer's spectrum rows (staged after the previous
        // reduction) and the next column have landed
        if constexpr (NB == 1) stage_wait<true>();
        const T *scur = sbuf + (NB == 2 ? cur : 0) * CMAX * QP;
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < Cs)
                mac_ws_dispatch<F, T, PPT, NW, false>(acc[c], v, scur + c * QP, off, (im_m >> c) & 1u,
                                                      (yo_m >> c) & 1u);
        if (n + 1 < n1) put_tail(cbuf + (cur ^ 1) * (N / 2), ny, tg, tail);
        if constexpr (NB == 2) {
            stage_wait<true>();
        } else {
            lds_barrier();   // every wave is past its reads of the spectrum rows
            if (n + 1 < n1) stage_spec(n + 1, 0);
        }
    }

    // every wave is past its last reads of the staged buffers: 2N words of
    // the group's area take the waves' inverse transforms
    T *cre = SH ? cw : gb;
    if constexpr (C::LANE) lane_twiddles<true>(ltw, tw, twlog, lane);
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        if (c < Cs) {
            ws_inverse_put<F, T, N, NW, L, PPT>(acc[c], xch, twp, twlog, lane, w, tws, cre, ltw);
            lds_barrier();
            if (un.active) {
                if (un.nyq)   // real partial column of the Nyquist unit
                    ws_store<T, N, NW, L, PPT, GT>(
                        cre, reinterpret_cast<cx<T> *>(Dny + (((size_t)un.split * B + un.b) * Ct + c) * (size_t)ldc),
                        tg, ny, 3);
                else
                    ws_store<T, N, NW, L, PPT, GT>(
                        cre, D + ((((size_t)un.split * B + un.b) * Ct + c) * M + un.u) * (size_t)ldc, tg, ny, un.part);
            }
            lds_barrier();
        }
    }
}

// Forward column pass of several observation levels at once (plans of up
// to three spectra): level j of the pass sees model layer n through
// spectral layer n + j (spec points at the pass's first level's window).
// One density column transform per layer serves all nlev levels, and the
// spectral layers form a ring of nlev + 1 in LDS: each step stages one new
// spectral layer (n + nlev) and one column, instead of nlev of each.
// Accumulator k = j * Cs + c (nlev * Cs <= 6) is written to slot k of D and
// Dny, whose slot stride is nlev * Cs.
template <typename T, int N>
__global__ void __launch_bounds__((WsCfg<T, N>::THREADS))
    __attribute__((amdgpu_waves_per_eu(WsCfg<T, N>::WAVES_PER_EU)))
    col_levels_ws_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec, cx<T> *__restrict__ D,
                         T *__restrict__ Dny, int B, int nz, int M, int ny, int ldc, int Cs, int nlev, int lps,
                         int nblk_ny, int Sny, int lps_ny, int nblk_main, unsigned imag_mask, unsigned yodd_mask,
                         const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N>;
    using F = typename C::FFT;
    constexpr int CMAX = 6;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    T *twq = lds;
    T *gb = lds + C::TWW + (size_t)g * C::group_words(CMAX);
    static_assert(C::spec_bufs(CMAX) == 2, "the spectral-layer ring takes both spectrum buffers");
    T *sbuf = gb;                                                        // ring: (nlev + 1) x Cs x QP <= 2 x CMAX x QP
    cx<T> *cbuf = reinterpret_cast<cx<T> *>(gb + 2 * CMAX * QP);         // 2 x N/2 complex
    T *xch = gb + 2 * CMAX * QP + 2 * C::CW + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);
    for (unsigned i = (unsigned)ny + tg; i < (unsigned)(N / 2); i += GT) {
        cbuf[i] = cx<T>{T(0), T(0)};
        cbuf[N / 2 + i] = cx<T>{T(0), T(0)};
    }

    WsTwiddles<T, N, PPT> tws;
    cx<T> cn[NW > 1 ? NW / 2 : 1];
    if constexpr (NW > 1) {
        tws.init(tw, twlog, lane, w);
        constexpr int LOGN = ilog2<N>::value;
#pragma unroll
        for (int n1 = 0; n1 < NW / 2; ++n1) cn[n1] = tw[(((unsigned)L * n1 * w) & (N - 1)) << (twlog - LOGN)];
    }
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<false>(ltw, tw, twlog, lane);

    const WsItem un = ws_item<GT, G>(g, M, B, nz, lps, nblk_ny, Sny, lps_ny, nblk_main);
    const unsigned row = spec_row(un.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const unsigned rowvals = (unsigned)Cs * QP;
    const int ring = nlev + 1;
    const int nk = nlev * Cs;
    const int n0 = un.n0;
    const int n1 = un.n1;

    cx<T> acc[CMAX][PPT];
#pragma unroll
    for (int k = 0; k < CMAX; ++k)
#pragma unroll
        for (int s = 0; s < PPT; ++s) acc[k][s] = cx<T>{T(0), T(0)};

    cx<T> tail{T(0), T(0)};
    auto stage_spec = [&](int sl) {
        stage_rows<T, GT, true>(spec + (size_t)sl * layer_vals + (size_t)row * rowvals,
                                sbuf + (size_t)(sl % ring) * rowvals, rowvals, tg);
    };
    if (n0 < n1) {
        for (int j = 0; j < nlev; ++j) stage_spec(n0 + j);
        stage_column<T, GT>(column(R, (size_t)un.b * nz + n0, M, un.u, ldc), cbuf, ny, tg, tail);
        put_tail(cbuf, ny, tg, tail);
    }
    stage_wait<true>();

    for (int n = n0; n < n1; ++n) {
        const int cur = (n - n0) & 1;
        if (n + 1 < n1) {
            stage_spec(n + nlev);
            stage_column<T, GT>(column(R, (size_t)un.b * nz + n + 1, M, un.u, ldc), cbuf + (cur ^ 1) * (N / 2), ny,
                                tg, tail);
        }
        cx<T> v[PPT];
        const cx<T> *xc = cbuf + cur * (N / 2);
        if (un.part == 0)
            form_z<F, T, N, NW, L, PPT, 0>(v, xc, lane, w, cn, tws);
        else if (un.part == 1)
            form_z<F, T, N, NW, L, PPT, 1>(v, xc, lane, w, cn, tws);
        else
            form_z<F, T, N, NW, L, PPT, 2>(v, xc, lane, w, cn, tws);
        ws_fft<false, F>(v, xch, lane, twp, twlog, ltw);
#pragma unroll
        for (int k = 0; k < CMAX; ++k)
            if (k < nk) {
                const int j = k / Cs, c = k - j * Cs;
                const T *srow = sbuf + (size_t)((n + j) % ring) * rowvals + (size_t)c * QP;
                mac_ws_dispatch<F, T, PPT, NW, false>(acc[k], v, srow, off, (imag_mask >> c) & 1u,
                                                      (yodd_mask >> c) & 1u);
            }
        if (n + 1 < n1) put_tail(cbuf + (cur ^ 1) * (N / 2), ny, tg, tail);
        stage_wait<true>();
    }

    T *cre = gb;
    if constexpr (C::LANE) lane_twiddles<true>(ltw, tw, twlog, lane);
#pragma unroll
    for (int k = 0; k < CMAX; ++k) {
        if (k < nk) {
            ws_inverse_put<F, T, N, NW, L, PPT>(acc[k], xch, twp, twlog, lane, w, tws, cre, ltw);
            lds_barrier();
            if (un.active) {
                if (un.nyq)
                    ws_store<T, N, NW, L, PPT, GT>(
                        cre, reinterpret_cast<cx<T> *>(Dny + (((size_t)un.split * B + un.b) * nk + k) * (size_t)ldc),
                        tg, ny, 3);
                else
                    ws_store<T, N, NW, L, PPT, GT>(
                        cre, D + ((((size_t)un.split * B + un.b) * nk + k) * M + un.u) * (size_t)ldc, tg, ny, un.part);
            }
            lds_barrier();
        }
    }
}

// Adjoint in the wave split: the Cs residual columns are staged and
// transformed once; per layer sum_c K^_{c,n} r^_c is inverse-transformed per
// wave and combined through LDS.
template <typename T, int N, int CMAX, int KIND>
__global__ void __launch_bounds__((WsCfg<T, N>::THREADS))
    __attribute__((amdgpu_waves_per_eu(WsCfg<T, N>::WAVES_PER_EU)))
    col_adjoint_ws_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec, cx<T> *__restrict__ Gout,
                          int B, int nz, int M, int ny, int ldc, int Cs, int Ct, int lps, int nblk_ny, int Sny,
                          int lps_ny, int nblk_main, unsigned imag_mask, unsigned yodd_mask,
                          const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    const unsigned im_m = KIND >= 0 ? (unsigned)(KIND & 0xFF) : imag_mask;
    const unsigned yo_m = KIND >= 0 ? (unsigned)((KIND >> 8) & 0xFF) : yodd_mask;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    constexpr int NB = C::spec_bufs(CMAX);
    // the Cs residual columns (setup only) fit the spectrum and combination areas
    static_assert(CMAX * N <= NB * CMAX * QP + 2 * C::CW, "residual columns exceed their staging area");
    T *twq = lds;
    T *gb = lds + C::TWW + (size_t)g * C::group_words(CMAX);
    T *sbuf = gb;                                                        // NB x CMAX x QP
    T *cre = gb + NB * CMAX * QP;                                        // combination: 2N words
    cx<T> *rbuf = reinterpret_cast<cx<T> *>(gb);                         // residual columns (setup only)
    T *xch = gb + NB * CMAX * QP + 2 * C::CW + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);

    WsTwiddles<T, N, PPT> tws;
    cx<T> cn[NW > 1 ? NW / 2 : 1];
    if constexpr (NW > 1) {
        tws.init(tw, twlog, lane, w);
        constexpr int LOGN = ilog2<N>::value;
#pragma unroll
        for (int n1 = 0; n1 < NW / 2; ++n1) cn[n1] = tw[(((unsigned)L * n1 * w) & (N - 1)) << (twlog - LOGN)];
    }
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<false>(ltw, tw, twlog, lane);

    const WsItem un = ws_item<GT, G>(g, M, B, nz, lps, nblk_ny, Sny, lps_ny, nblk_main);
    const unsigned row = spec_row(un.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const int n0 = un.n0;
    const int n1 = un.n1;

    // residual columns into the spectrum (and, with one spectrum buffer, the
    // combination) area
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
        if (c < Cs) {
            for (unsigned i = (unsigned)ny + tg; i < (unsigned)(N / 2); i += GT) rbuf[c * (N / 2) + i] = cx<T>{T(0), T(0)};
            cx<T> tail{T(0), T(0)};
            stage_column<T, GT>(column(R, (size_t)un.b * Ct + c, M, un.u, ldc), rbuf + c * (N / 2), ny, tg, tail);
            put_tail(rbuf + c * (N / 2), ny, tg, tail);
        }
    }
    stage_wait<true>();
    cx<T> rh[CMAX][PPT];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
#pragma unroll
        for (int s = 0; s < PPT; ++s) rh[c][s] = cx<T>{T(0), T(0)};
        if (c < Cs) {
            const cx<T> *xc = rbuf + c * (N / 2);
            if (un.part == 0)
                form_z<F, T, N, NW, L, PPT, 0>(rh[c], xc, lane, w, cn, tws);
            else if (un.part == 1)
                form_z<F, T, N, NW, L, PPT, 1>(rh[c], xc, lane, w, cn, tws);
            else
                form_z<F, T, N, NW, L, PPT, 2>(rh[c], xc, lane, w, cn, tws);
            ws_fft<false, F>(rh[c], xch, lane, twp, twlog, ltw);
        }
    }
    lds_barrier();   // every wave is past its reads of the residual columns
    if constexpr (C::LANE) lane_twiddles<true>(ltw, tw, twlog, lane);

    if (n0 < n1) stage_rows<T, GT, true>(spec + (size_t)n0 * layer_vals + (size_t)row * Cs * QP, sbuf, (unsigned)Cs * QP, tg);
    stage_wait<true>();

    for (int n = n0; n < n1; ++n) {
        const int cur = (n - n0) & 1;
        if constexpr (NB == 2) {
            if (n + 1 < n1)
                stage_rows<T, GT, true>(spec + (size_t)(n + 1) * layer_vals + (size_t)row * Cs * QP,
                                        sbuf + (cur ^ 1) * CMAX * QP, (unsigned)Cs * QP, tg);
        }
        const T *scur = sbuf + (NB == 2 ? cur : 0) * CMAX * QP;
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) v[s] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < Cs)
                mac_ws_dispatch<F, T, PPT, NW, true>(v, rh[c], scur + c * QP, off, (im_m >> c) & 1u,
                                                     (yo_m >> c) & 1u);
        if constexpr (NB == 1) {
            // one buffer: the next layer's rows stream in during this
            // layer's inverse transform, once every wave is past its reads
            lds_barrier();
            if (n + 1 < n1)
                stage_rows<T, GT, true>(spec + (size_t)(n + 1) * layer_vals + (size_t)row * Cs * QP, sbuf,
                                        (unsigned)Cs * QP, tg);
        }
        ws_inverse_put<F, T, N, NW, L, PPT>(v, xch, twp, twlog, lane, w, tws, cre, ltw);
        lds_barrier();
        if (un.active)
            ws_store<T, N, NW, L, PPT, GT>(cre, Gout + (((size_t)un.b * nz + n) * M + un.u) * (size_t)ldc, tg, ny,
                                           un.part);
        stage_wait<true>();
    }
}

// Adjoint column pass of several observation levels at once (plans of up
// to three spectra): the nlev * Cs residual columns of the pass's levels
// (R slot k = j * Cs + c: level j, spectrum c) are transformed once; per
// model layer n, sum_{j,c} K^_{c,n+j} r^_{j,c} is inverse-transformed into
// Gout column n.  Spectral layers form a ring of nlev + 1 in LDS as in the
// forward levels pass.
template <typename T, int N>
__global__ void __launch_bounds__((WsCfg<T, N>::THREADS))
    __attribute__((amdgpu_waves_per_eu(WsCfg<T, N>::WAVES_PER_EU)))
    col_levels_adjoint_ws_kernel(const cx<T> *__restrict__ R, const T *__restrict__ spec, cx<T> *__restrict__ Gout,
                                 int B, int nz, int M, int ny, int ldc, int Cs, int nlev, int lps, int nblk_ny,
                                 int Sny, int lps_ny, int nblk_main, unsigned imag_mask, unsigned yodd_mask,
                                 const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N>;
    using F = typename C::FFT;
    constexpr int CMAX = 6;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    T *twq = lds;
    T *gb = lds + C::TWW + (size_t)g * C::group_words(CMAX);
    static_assert(C::spec_bufs(CMAX) == 2, "the spectral-layer ring takes both spectrum buffers");
    T *sbuf = gb;                                                        // ring: (nlev + 1) x Cs x QP <= 2 x CMAX x QP
    T *cre = gb + 2 * CMAX * QP;                                         // combination: 2N words
    cx<T> *rbuf = reinterpret_cast<cx<T> *>(gb);                         // residual columns (setup only)
    T *xch = gb + 2 * CMAX * QP + 2 * C::CW + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);

    WsTwiddles<T, N, PPT> tws;
    cx<T> cn[NW > 1 ? NW / 2 : 1];
    if constexpr (NW > 1) {
        tws.init(tw, twlog, lane, w);
        constexpr int LOGN = ilog2<N>::value;
#pragma unroll
        for (int n1 = 0; n1 < NW / 2; ++n1) cn[n1] = tw[(((unsigned)L * n1 * w) & (N - 1)) << (twlog - LOGN)];
    }
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<false>(ltw, tw, twlog, lane);

    const WsItem un = ws_item<GT, G>(g, M, B, nz, lps, nblk_ny, Sny, lps_ny, nblk_main);
    const unsigned row = spec_row(un.uv, (unsigned)M);
    const size_t layer_vals = (size_t)(M + 1) * Cs * QP;
    const unsigned rowvals = (unsigned)Cs * QP;
    const int ring = nlev + 1;
    const int nk = nlev * Cs;
    const int n0 = un.n0;
    const int n1 = un.n1;

    // residual columns into the spectrum area (nk x N/2 complex fit in 2 x CMAX x QP words)
#pragma unroll
    for (int k = 0; k < CMAX; ++k) {
        if (k < nk) {
            for (unsigned i = (unsigned)ny + tg; i < (unsigned)(N / 2); i += GT) rbuf[k * (N / 2) + i] = cx<T>{T(0), T(0)};
            cx<T> tail{T(0), T(0)};
            stage_column<T, GT>(column(R, (size_t)un.b * nk + k, M, un.u, ldc), rbuf + k * (N / 2), ny, tg, tail);
            put_tail(rbuf + k * (N / 2), ny, tg, tail);
        }
    }
    stage_wait<true>();
    cx<T> rh[CMAX][PPT];
#pragma unroll
    for (int k = 0; k < CMAX; ++k) {
#pragma unroll
        for (int s = 0; s < PPT; ++s) rh[k][s] = cx<T>{T(0), T(0)};
        if (k < nk) {
            const cx<T> *xc = rbuf + k * (N / 2);
            if (un.part == 0)
                form_z<F, T, N, NW, L, PPT, 0>(rh[k], xc, lane, w, cn, tws);
            else if (un.part == 1)
                form_z<F, T, N, NW, L, PPT, 1>(rh[k], xc, lane, w, cn, tws);
            else
                form_z<F, T, N, NW, L, PPT, 2>(rh[k], xc, lane, w, cn, tws);
            ws_fft<false, F>(rh[k], xch, lane, twp, twlog, ltw);
        }
    }
    lds_barrier();   // every wave is past its reads of the residual columns
    if constexpr (C::LANE) lane_twiddles<true>(ltw, tw, twlog, lane);

    auto stage_spec = [&](int sl) {
        stage_rows<T, GT, true>(spec + (size_t)sl * layer_vals + (size_t)row * rowvals,
                                sbuf + (size_t)(sl % ring) * rowvals, rowvals, tg);
    };
    if (n0 < n1)
        for (int j = 0; j < nlev; ++j) stage_spec(n0 + j);
    stage_wait<true>();

    for (int n = n0; n < n1; ++n) {
        if (n + 1 < n1) stage_spec(n + nlev);
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) v[s] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int k = 0; k < CMAX; ++k)
            if (k < nk) {
                const int j = k / Cs, c = k - j * Cs;
                const T *srow = sbuf + (size_t)((n + j) % ring) * rowvals + (size_t)c * QP;
                mac_ws_dispatch<F, T, PPT, NW, true>(v, rh[k], srow, off, (imag_mask >> c) & 1u,
                                                     (yodd_mask >> c) & 1u);
            }
        ws_inverse_put<F, T, N, NW, L, PPT>(v, xch, twp, twlog, lane, w, tws, cre, ltw);
        lds_barrier();
        if (un.active)
            ws_store<T, N, NW, L, PPT, GT>(cre, Gout + (((size_t)un.b * nz + n) * M + un.u) * (size_t)ldc, tg, ny,
                                           un.part);
        stage_wait<true>();
    }
}

// ---------------------------------------------------------------------------
// Observation levels as a Toeplitz product in depth (the equal-dimension
// survey: eq. 10-11 and the block matrix after eq. 22).
//
// Level t of the forward operator is d^_{t,c}(k) = sum_n conj(K^_{c,n+t}(k))
// rho^_n(k): at each frequency a Toeplitz product along depth.  Instead of a
// column pass per level (each re-reading the density and nz spectral
// layers), three steps run once each:
//   col_spectra_ws_kernel   y-transform of every column into its spectrum
//   levels_*_toeplitz_kernel the depth products of a block of levels at
//                           each frequency, every spectral layer of the
//                           block's window read once
//   col_inverse_ws_kernel   inverse y-transform of every output spectrum
// The adjoint runs the same steps with levels and layers exchanged:
// g^_n(k) = sum_t sum_c K^_{c,n+t}(k) r^_{t,c}(k).
//
// A column's spectrum (ky in [0, N)) is stored as two rows of QP values in
// the order of the resident spectrum rows: row 0 holds ky = q at spec_pos(q)
// for q in [0, N/2), row 1 holds ky = N - q at spec_pos(q) for q in [1, N/2],
// so that a component's resident quarter-plane row gives K^ for both rows
// at the same position (with the component's y-parity sign on row 1).
// Entries no frequency maps to are neither written nor read as data.  A
// slab is [M+1 rows in spec_row order][2][QP] complex values.

// Work of one group of the transform kernels: virtual unit uv of model b;
// the block's groups share the slab range (blockIdx.y), so every group of a
// block runs the same number of workgroup barriers.
struct SpItem {
    unsigned uv, u, b;
    int part;
    bool active;
};

template <int G>
__device__ __forceinline__ SpItem sp_item(unsigned g, int M, int B)
{
    SpItem it;
    const unsigned U1 = (unsigned)M + 1;
    const unsigned gi = blockIdx.x * G + g;
    it.active = gi < U1 * (unsigned)B;
    const unsigned gc = it.active ? gi : 0u;
    it.uv = __builtin_amdgcn_readfirstlane(gc % U1);
    it.b = __builtin_amdgcn_readfirstlane(gc / U1);
    it.u = it.uv == (unsigned)M ? 0u : it.uv;
    it.part = it.uv == 0 ? 1 : (it.uv == (unsigned)M ? 2 : 0);
    return it;
}

// Offset of slot s's frequency in a two-row spectrum (see above): row 0 at
// the lower slots' resident positions, row 1 at QP + the upper slots'.
template <typename F, int PPT, int QP>
__device__ __forceinline__ unsigned sp_offset(int s, const unsigned (&off)[PPT])
{
    const bool upper = F::elem_out(s) >= PPT / 2;
    return upper ? (unsigned)QP + off[s] : off[s];
}

// Spectra of the columns of slabs [s0, s1) (s0, s1 from blockIdx.y and
// `chunk`) of every model: X[b * nsrc + s] from the columns of
// R[b * nsrc + s] (laid out [slab][M][ldc]).
template <typename T, int N>
__global__ void __launch_bounds__((WsCfg<T, N>::THREADS))
    col_spectra_ws_kernel(const cx<T> *__restrict__ R, cx<T> *__restrict__ X, int B, int nsrc, int M, int ny,
                          int ldc, int chunk, const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    constexpr int GW = 2 * C::CW + NW * C::XW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    T *twq = lds;
    T *gb = lds + C::TWW + (size_t)g * GW;
    cx<T> *cbuf = reinterpret_cast<cx<T> *>(gb);                        // 2 x N/2 complex
    T *xch = gb + 2 * C::CW + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);
    for (unsigned i = (unsigned)ny + tg; i < (unsigned)(N / 2); i += GT) {
        cbuf[i] = cx<T>{T(0), T(0)};
        cbuf[N / 2 + i] = cx<T>{T(0), T(0)};
    }
    WsTwiddles<T, N, PPT> tws;
    cx<T> cn[NW > 1 ? NW / 2 : 1];
    if constexpr (NW > 1) {
        tws.init(tw, twlog, lane, w);
        constexpr int LOGN = ilog2<N>::value;
#pragma unroll
        for (int n1 = 0; n1 < NW / 2; ++n1) cn[n1] = tw[(((unsigned)L * n1 * w) & (N - 1)) << (twlog - LOGN)];
    }
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<false>(ltw, tw, twlog, lane);

    const SpItem it = sp_item<G>(g, M, B);
    const unsigned row = spec_row(it.uv, (unsigned)M);
    const int s0 = (int)blockIdx.y * chunk;
    const int s1 = min(nsrc, s0 + chunk);
    cx<T> tail{T(0), T(0)};
    auto stage_col = [&](int sl, int buf) {
        stage_column<T, GT>(column(R, (size_t)it.b * nsrc + sl, M, it.u, ldc), cbuf + buf * (N / 2), ny, tg, tail);
    };
    if (s0 < s1) {
        stage_col(s0, 0);
        put_tail(cbuf, ny, tg, tail);
    }
    stage_wait<true>();
    for (int sl = s0; sl < s1; ++sl) {
        const int cur = (sl - s0) & 1;
        if (sl + 1 < s1) stage_col(sl + 1, cur ^ 1);
        cx<T> v[PPT];
        const cx<T> *xc = cbuf + cur * (N / 2);
        if (it.part == 0)
            form_z<F, T, N, NW, L, PPT, 0>(v, xc, lane, w, cn, tws);
        else if (it.part == 1)
            form_z<F, T, N, NW, L, PPT, 1>(v, xc, lane, w, cn, tws);
        else
            form_z<F, T, N, NW, L, PPT, 2>(v, xc, lane, w, cn, tws);
        ws_fft<false, F>(v, xch, lane, twp, twlog, ltw);
        if (it.active) {
            cx<T> *dst = X + (((size_t)it.b * nsrc + sl) * (M + 1) + row) * (2 * QP);
#pragma unroll
            for (int s = 0; s < PPT; ++s) dst[sp_offset<F, PPT, QP>(s, off)] = v[s];
        }
        if (sl + 1 < s1) put_tail(cbuf + (cur ^ 1) * (N / 2), ny, tg, tail);
        stage_wait<true>();
    }
}

// Inverse of col_spectra_ws_kernel: the columns of D[b * nsrc + s] (laid out
// [slab][M][ldc], y < ny written; the two real bins into the fields of
// packed unit 0) from the spectra X[b * nsrc + s].
template <typename T, int N>
__global__ void __launch_bounds__((WsCfg<T, N>::THREADS))
    col_inverse_ws_kernel(const cx<T> *__restrict__ X, cx<T> *__restrict__ D, int B, int nsrc, int M, int ny,
                          int ldc, int chunk, const cx<T> *__restrict__ tw, int twlog)
{
    using C = WsCfg<T, N>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, L = C::L, NW = C::NW, G = C::G, GT = C::GT, QP = C::QP;
    constexpr int GW = 2 * N + NW * C::XW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned g = wv / NW, w = wv % NW;
    const unsigned tg = threadIdx.x - g * GT;
    T *twq = lds;
    T *gb = lds + C::TWW + (size_t)g * GW;
    T *cre = gb;                                                        // combination: 2N words
    T *xch = gb + 2 * N + w * C::XW;
    const cx<T> *twp = reinterpret_cast<const cx<T> *>(twq);
    F::load_stage_table(twq, tw, twlog, threadIdx.x, C::THREADS);
    WsTwiddles<T, N, PPT> tws;
    if constexpr (NW > 1) tws.init(tw, twlog, lane, w);
    unsigned off[PPT];   // this lane's slots in a resident spectrum row
    ws_spec_offsets<F, PPT, NW, L>(off, lane, w);
    cx<T> ltw[C::LANE ? 9 : 1];
    if constexpr (C::LANE) lane_twiddles<true>(ltw, tw, twlog, lane);
    __syncthreads();   // stage table

    const SpItem it = sp_item<G>(g, M, B);
    const unsigned row = spec_row(it.uv, (unsigned)M);
    const int s0 = (int)blockIdx.y * chunk;
    const int s1 = min(nsrc, s0 + chunk);
    for (int sl = s0; sl < s1; ++sl) {
        const cx<T> *src = X + (((size_t)it.b * nsrc + sl) * (M + 1) + row) * (2 * QP);
        cx<T> v[PPT];
#pragma unroll
        for (int s = 0; s < PPT; ++s) v[s] = src[sp_offset<F, PPT, QP>(s, off)];
        ws_inverse_put<F, T, N, NW, L, PPT>(v, xch, twp, twlog, lane, w, tws, cre, ltw);
        lds_barrier();
        if (it.active)
            ws_store<T, N, NW, L, PPT, GT>(cre, D + (((size_t)it.b * nsrc + sl) * M + it.u) * (size_t)ldc, tg, ny,
                                           it.part);
        lds_barrier();
    }
}

constexpr int kToepThreads = 256;

// Block of a depth-product launch: blocks are dealt to the eight XCDs in
// turn, and the output blocks of one position tile go to the same XCD back
// to back, so that they meet its inputs and spectral layers in one L2.
// Returns false for the padding blocks of the last round.
struct ToepBlock {
    unsigned tile, row, zb;
};

__device__ __forceinline__ bool toep_block(int ntile, int M, int nzb, ToepBlock &tb)
{
    const unsigned lb = blockIdx.x, xcd = lb & 7u, k = lb >> 3;
    const unsigned zb = k % (unsigned)nzb, tgl = (k / (unsigned)nzb) * 8u + xcd;
    if (tgl >= (unsigned)ntile * ((unsigned)M + 1u)) return false;
    tb.tile = tgl % (unsigned)ntile;
    tb.row = tgl / (unsigned)ntile;
    tb.zb = zb;
    return true;
}

// Depth products of the observation levels at one tile of 32 positions of
// one spectrum row (lane l: position tile * 32 + l % 32, row l / 32 of the
// two-row spectrum) of one model (blockIdx.y).  Forward: each wave owns TL
// consecutive levels o of one component c,
//   out[b][o][c] = sum_n conj(K^_{c, o + n}) X[b][n],  n < nz;
// adjoint: each wave owns TL consecutive layers n,
//   out[b][n] (+)= sum_c sum_t K^_{c, n + t} X[b][t][c],  t < nlev.
// K^ comes from the window `spec` of nz + nlev - 1 spectral layers
// ([layer][M+1 rows][Cs][QP], resident order).  The inputs pass through LDS
// in chunks of JC, and the spectral values of the block's outputs through a
// ring of KRING layers of the tile (a chunk adds JC layers to it); the next
// chunk's inputs and layers are loaded into registers while this chunk is
// computed.  Each thread slides its TL spectral values one layer per input,
// so a step is one LDS read of an input, one of a spectral value and TL
// complex multiply-adds.  Forward outputs are [B][nlev][Ct][rows][2][QP]
// and adjoint inputs likewise (offset by the caller to a group's first
// component); adjoint outputs [B][nz][rows][2][QP].
constexpr int kToepJC = 16;

#ifndef GF_TOEP_TL64
#define GF_TOEP_TL64 8
#endif
#ifndef GF_TOEP_TL32
#define GF_TOEP_TL32 16
#endif
#ifndef GF_TOEP_WPE
#define GF_TOEP_WPE 4
#endif
template <typename T>
constexpr int toep_tl()
{
    return sizeof(T) == 8 ? GF_TOEP_TL64 : GF_TOEP_TL32;
}

template <typename T, int TL>
constexpr size_t toep_lds_bytes()
{
    return (size_t)((kToepThreads / 64) * TL + kToepJC) * 32 * sizeof(T) + (size_t)kToepJC * 64 * sizeof(cx<T>);
}

template <typename T, int TL, bool ADJ>
__global__ void __launch_bounds__(kToepThreads) __attribute__((amdgpu_waves_per_eu(GF_TOEP_WPE)))
    levels_toeplitz_kernel(const cx<T> *__restrict__ X, const T *__restrict__ spec, cx<T> *__restrict__ out,
                           int nz, int nlev, int M, int QP, int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask,
                           int ntile, int nzb, int accumulate)
{
    constexpr int NWV = kToepThreads / 64, JC = kToepJC;
    constexpr int KRING = NWV * TL + JC;                 // layers of the tile held in LDS
    constexpr int KPT = (JC * 32 + kToepThreads - 1) / kToepThreads;   // new spectral values per thread and chunk
    constexpr int XPT = JC * 64 / kToepThreads;          // inputs per thread and chunk
    static_assert(JC % TL == 0 && XPT * kToepThreads == JC * 64, "chunk shape");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *ks = reinterpret_cast<T *>(smem_raw);                            // [KRING][32]
    cx<T> *xs = reinterpret_cast<cx<T> *>(smem_raw + (size_t)KRING * 32 * sizeof(T));   // [JC][64]
    ToepBlock tb;
    if (!toep_block(ntile, M, nzb, tb)) return;
    const unsigned lane = threadIdx.x & 63u, l32 = lane & 31u;
    const int wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned U1 = (unsigned)M + 1;
    const unsigned tile = tb.tile, row = tb.row;
    const unsigned b = blockIdx.y;
    const unsigned half = lane >> 5;
    const unsigned pos = tile * 32u + l32;
    const int nwin = nz + nlev - 1;
    const size_t kstride = (size_t)U1 * Cs * QP;                        // one spectral layer
    const int nzb_c = ADJ ? nzb : nzb / Cs;
    const int c_fwd = ADJ ? 0 : (int)tb.zb / nzb_c;
    const int o_blk = (int)(tb.zb % (unsigned)nzb_c) * NWV * TL;   // first output of the block
    const int nout = ADJ ? nz : nlev;
    const int nin = ADJ ? nlev : nz;
    const int o0 = o_blk + wave * TL;

    // Staged elements of this thread: spectral values e = threadIdx.x + i *
    // threads of a chunk's JC new layers (layer e / 32, position e % 32) and
    // inputs e = threadIdx.x + i * threads (input e / 64, slot e % 64); the
    // position and slot do not depend on i (threads is a multiple of 64).
    const unsigned kp32 = min(tile * 32u + (threadIdx.x & 31u), (unsigned)QP - 1u);
    const unsigned xsl = threadIdx.x & 63u, xp32 = tile * 32u + (xsl & 31u);
    const bool xok = xp32 < (unsigned)QP;
    const size_t xslab = (size_t)U1 * 2 * QP;                          // one input slab (values)
    // spectral value of layer o_blk + r at this thread's position (clamped into the window)
    auto kval = [&](const T *kc, int r) -> T { return kc[(size_t)min(o_blk + r, nwin - 1) * kstride]; };
    // input j of this thread's slot, times the factor that turns the real k of
    // the resident spectrum into the product: forward conj(K^) x, adjoint K^ x,
    // with K^ = k (real component) or i k (imaginary), and k negated on row 1
    // for a component odd in y
    auto xval = [&](const cx<T> *xc, size_t jstride, int j, bool im, bool neg) -> cx<T> {
        T vr = T(0), vi = T(0);
        if (j < nin && xok) {
            const T *src = reinterpret_cast<const T *>(xc + (size_t)j * jstride);
            vr = src[0];
            vi = src[1];
        }
        if (im) {
            const T t = vr;
            vr = ADJ ? -vi : vi;
            vi = ADJ ? t : -t;
        }
        if (neg) {
            vr = -vr;
            vi = -vi;
        }
        return cx<T>{vr, vi};
    };
    constexpr int XROWS = kToepThreads / 64;   // inputs staged per pass of the threads

    cx<T> acc[TL];
#pragma unroll
    for (int i = 0; i < TL; ++i) acc[i] = cx<T>{T(0), T(0)};
    const bool active = o0 < nout;   // waves past the last output only stage and wait
    const int cbeg = ADJ ? 0 : c_fwd, cend = ADJ ? Cs : c_fwd + 1;
    for (int c = cbeg; c < cend; ++c) {
        const bool im = (imag_mask >> c) & 1u, neg = (xsl >> 5) && ((yodd_mask >> c) & 1u);
        const T *kc = spec + ((size_t)row * Cs + c) * QP + kp32;
        // this thread's slot of input 0 and the stride between inputs
        const cx<T> *xc = X + (ADJ ? ((size_t)b * nlev * Ct + c) : (size_t)b * nz) * xslab +
                          ((size_t)row * 2 + (xsl >> 5)) * QP + xp32;
        const size_t jstride = ADJ ? (size_t)Ct * xslab : xslab;
        const int kr0 = (int)(threadIdx.x >> 5), krs = kToepThreads / 32;
        const int xr0 = (int)(threadIdx.x >> 6);
        __syncthreads();   // every wave is past its reads of the previous component's buffers
        // the ring's first KRING - 1 layers and the first chunk of inputs
        for (int r = kr0; r < KRING - 1; r += krs) ks[r * 32 + (int)(threadIdx.x & 31u)] = kval(kc, r);
#pragma unroll
        for (int i = 0; i < XPT; ++i) xs[threadIdx.x + i * kToepThreads] = xval(xc, jstride, xr0 + i * XROWS, im, neg);
        __syncthreads();
        T win[TL];
#pragma unroll
        for (int i = 0; i < TL - 1; ++i) win[i] = ks[(wave * TL + i) * 32 + l32];
        int slot = wave * TL + TL - 1;   // ring slot of the layer the next step adds (< KRING)
        for (int j0 = 0; j0 < nin; j0 += JC) {
            const bool next = j0 + JC < nin;
            // the next chunk's inputs and its JC new layers (relative layers
            // j0 + KRING - 1 ...), into registers
            cx<T> xp[XPT];
            T kp[KPT];
            if (next) {
#pragma unroll
                for (int i = 0; i < XPT; ++i) xp[i] = xval(xc, jstride, j0 + JC + xr0 + i * XROWS, im, neg);
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const int r = kr0 + i * krs;
                    kp[i] = r < JC ? kval(kc, j0 + KRING - 1 + r) : T(0);
                }
            }
            if (active) {
#pragma unroll 1
                for (int jj = 0; jj < JC; jj += TL) {
#pragma unroll
                    for (int r = 0; r < TL; ++r) {
                        win[(r + TL - 1) % TL] = ks[slot * 32 + (int)l32];
                        slot = slot + 1 == KRING ? 0 : slot + 1;
                        const cx<T> x = xs[(jj + r) * 64 + (int)lane];
#pragma unroll
                        for (int i = 0; i < TL; ++i) {
                            const T k = win[(r + i) % TL];
                            acc[i].re += k * x.re;
                            acc[i].im += k * x.im;
                        }
                    }
                }
            }
            if (next) {
                __syncthreads();   // every wave is past its reads of this chunk
#pragma unroll
                for (int i = 0; i < XPT; ++i) xs[threadIdx.x + i * kToepThreads] = xp[i];
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const int r = kr0 + i * krs;
                    if (r < JC) ks[((j0 + KRING - 1 + r) % KRING) * 32 + (int)(threadIdx.x & 31u)] = kp[i];
                }
                __syncthreads();
            }
        }
    }
    if (pos < (unsigned)QP) {
#pragma unroll
        for (int i = 0; i < TL; ++i) {
            const int o = o0 + i;
            if (o < nout) {
                const size_t slab = ADJ ? (size_t)b * nz + o : ((size_t)b * nlev + o) * Ct + c_fwd;
                cx<T> *dst = out + ((slab * U1 + row) * 2 + half) * (size_t)QP + pos;
                cx<T> v = acc[i];
                if (ADJ && accumulate) v = add(*dst, v);
                *dst = v;
            }
        }
    }
}

// Plan time: full-length column FFT of the row-transformed kernel fields
// (double), keeping one real per frequency of the quarter plane.  Virtual
// units as in the adjoint.
template <typename TO, int N>
__global__ void __launch_bounds__((ColCfg<double, N>::THREADS))
    col_kgen_kernel(const cx<double> *__restrict__ Rk, TO *__restrict__ spec, int nl, int n0, int Cs,
                    int nz, int M, unsigned imag_mask, unsigned yodd_mask, const cx<double> *__restrict__ tw,
                    int twlog)
{
    using C = ColCfg<double, N>;
    using F = typename C::FFTK;
    constexpr int PPT = C::PPT, NT = C::NT, G = C::G, W = F::lds_words();
    constexpr unsigned QPO = ColCfg<TO, N>::QP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    double *sre = lds + (size_t)g * 2 * W;
    double *sim = sre + W;

    const unsigned U1 = M + 1;
    const unsigned npair = (unsigned)(nl * Cs);
    const unsigned gi = blockIdx.x * G + g;
    const bool active = gi < npair * U1;
    const unsigned pair = active ? gi / U1 : 0;
    const unsigned uv = active ? gi % U1 : 0;
    const unsigned u = (uv == (unsigned)M) ? 0u : uv;
    const int part = uv == 0 ? 1 : (uv == (unsigned)M ? 2 : 0);
    const int c = (int)(pair % Cs);
    const int n = n0 + (int)(pair / Cs);

    cx<double> v[PPT];
    const cx<double> *col = column(Rk, pair, M, u, N);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const unsigned y = t + NT * F::elem_in(s);
        cx<double> x = active ? col[y] : cx<double>{0.0, 0.0};
        if (part == 1) x.im = 0.0;
        if (part == 2) x = cx<double>{x.im, 0.0};
        v[s] = x;
    }
    F::template run<false>(v, sre, sim, t, tw, twlog);
    if (active) {
        const bool im = (imag_mask >> c) & 1u;
        const bool yo = (yodd_mask >> c) & 1u;
        TO *dst = spec + (((size_t)n * U1 + spec_row(uv, M)) * Cs + c) * QPO;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const unsigned ky = t + NT * F::elem_out(s);
            // a component odd in y has an exactly zero spectrum at ky = Py/2
            // (its terms at +-b cancel and b = Py/2 is padding); store the
            // zero rather than the transform's rounding residue
            if (ky <= N / 2) dst[spec_pos<TO, N>(ky)] = (yo && ky == N / 2) ? TO(0) : (TO)(im ? v[s].im : v[s].re);
        }
        // zero the row padding so staged blocks hold no stale values
        if (t < QPO - (N / 2 + 1)) dst[N / 2 + 1 + t] = TO(0);
    }
}

template <typename T, int N, int CMAX, int KIND, bool SH>
static int run_fwd_ws(const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc, int Cs,
                      int Ct, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask, unsigned yodd_mask,
                      const void *tw, int twlog, hipStream_t st)
{
    using C = WsCfg<T, N, SH>;
    const long nbb = (B + C::G - 1) / C::G;
    const long nblk_main = SH ? (long)M * nbb : ((long)M * B + C::G - 1) / C::G;
    const long nblk_ny = (long)nq.Sny * nbb;
    const size_t lds = C::lds_bytes(CMAX);
    if (lds > lds_limit()) return -3;
    if (nq.Sny < 1 || nq.lps_ny < 1 || !nq.Dny) return -2;
    hipLaunchKernelGGL((col_forward_ws_kernel<T, N, CMAX, KIND, SH>), dim3((unsigned)(nblk_ny + nsplit * nblk_main)),
                       dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)D,
                       (T *)nq.Dny, B, nz, M, ny, ldc, Cs, Ct, lps, (int)nblk_ny, nq.Sny, nq.lps_ny,
                       (int)nblk_main, imag_mask, yodd_mask, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int N, int CMAX, int KIND>
static int run_fwd(const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc, int Cs,
                   int Ct, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask, unsigned yodd_mask,
                   const void *tw, int twlog, hipStream_t st)
{
    if constexpr (use_ws<N>()) {
        if constexpr (ws_shared_exists<T, N>())
            if (ws_shared_for<T, N>(B))
                return run_fwd_ws<T, N, CMAX, KIND, true>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq,
                                                          imag_mask, yodd_mask, tw, twlog, st);
        return run_fwd_ws<T, N, CMAX, KIND, false>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq,
                                                   imag_mask, yodd_mask, tw, twlog, st);
    } else {
        using C = ColCfg<T, N>;
        const long groups = (long)(M + 1) * B;
        const long nblk = (groups + C::G - 1) / C::G;
        const size_t lds = C::lds_bytes(CMAX, true);
        if (lds > lds_limit()) return -3;
        hipLaunchKernelGGL((col_forward_kernel<T, N, CMAX, KIND>), dim3((unsigned)nblk, (unsigned)nsplit),
                           dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)D,
                           B, nz, M, ny, ldc, Cs, Ct, lps, imag_mask, yodd_mask, (const cx<T> *)tw, twlog);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
}

template <typename T, int N, int CMAX, int KIND>
static int run_adj(const void *R, const void *spec, void *Gout, int B, int nz, int M, int ny, int ldc, int Cs,
                   int Ct, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask, unsigned yodd_mask,
                   const void *tw, int twlog, hipStream_t st)
{
    if constexpr (use_ws<N>()) {
        // the adjoint keeps one item per group: its Cs transformed residual
        // columns stay in registers across the layers, which leaves no room
        // for the extra resident waves of the shared layout
        using C = WsCfg<T, N>;
        const long nblk_main = ((long)M * B + C::G - 1) / C::G;
        const long nblk_ny = (long)nq.Sny * ((B + C::G - 1) / C::G);
        const size_t lds = C::lds_bytes(CMAX);
        if (lds > lds_limit()) return -3;
        if (nq.Sny < 1 || nq.lps_ny < 1) return -2;
        hipLaunchKernelGGL((col_adjoint_ws_kernel<T, N, CMAX, KIND>), dim3((unsigned)(nblk_ny + nsplit * nblk_main)),
                           dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)Gout, B, nz,
                           M, ny, ldc, Cs, Ct, lps, (int)nblk_ny, nq.Sny, nq.lps_ny, (int)nblk_main, imag_mask,
                           yodd_mask, (const cx<T> *)tw, twlog);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    } else {
        using C = ColCfg<T, N>;
        const long groups = (long)(M + 1) * B;
        const long nblk = (groups + C::G - 1) / C::G;
        const size_t lds = C::lds_bytes(CMAX, false);
        if (lds > lds_limit()) return -3;
        hipLaunchKernelGGL((col_adjoint_kernel<T, N, CMAX, KIND>), dim3((unsigned)nblk, (unsigned)nsplit),
                           dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec,
                           (cx<T> *)Gout, B, nz, M, ny, ldc, Cs, Ct, lps, imag_mask, yodd_mask,
                           (const cx<T> *)tw, twlog);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
}

template <typename T, int N>
static int run_levels(const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc, int Cs,
                      int nlev, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask, unsigned yodd_mask,
                      const void *tw, int twlog, hipStream_t st)
{
    if constexpr (use_ws<N>()) {
        using C = WsCfg<T, N>;
        const long nblk_main = ((long)M * B + C::G - 1) / C::G;
        const long nblk_ny = (long)nq.Sny * ((B + C::G - 1) / C::G);
        const size_t lds = C::lds_bytes(6);
        if (lds > lds_limit()) return -3;
        if (nq.Sny < 1 || nq.lps_ny < 1 || !nq.Dny) return -2;
        hipLaunchKernelGGL((col_levels_ws_kernel<T, N>), dim3((unsigned)(nblk_ny + nsplit * nblk_main)),
                           dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)D,
                           (T *)nq.Dny, B, nz, M, ny, ldc, Cs, nlev, lps, (int)nblk_ny, nq.Sny, nq.lps_ny,
                           (int)nblk_main, imag_mask, yodd_mask, (const cx<T> *)tw, twlog);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    } else {
        return -2;
    }
}

template <typename T, int N>
static int run_levels_adj(const void *R, const void *spec, void *Gout, int B, int nz, int M, int ny, int ldc, int Cs,
                          int nlev, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask, unsigned yodd_mask,
                          const void *tw, int twlog, hipStream_t st)
{
    if constexpr (use_ws<N>()) {
        using C = WsCfg<T, N>;
        const long nblk_main = ((long)M * B + C::G - 1) / C::G;
        const long nblk_ny = (long)nq.Sny * ((B + C::G - 1) / C::G);
        const size_t lds = C::lds_bytes(6);
        if (lds > lds_limit()) return -3;
        if (nq.Sny < 1 || nq.lps_ny < 1) return -2;
        hipLaunchKernelGGL((col_levels_adjoint_ws_kernel<T, N>), dim3((unsigned)(nblk_ny + nsplit * nblk_main)),
                           dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)Gout, B, nz, M,
                           ny, ldc, Cs, nlev, lps, (int)nblk_ny, nq.Sny, nq.lps_ny, (int)nblk_main, imag_mask,
                           yodd_mask, (const cx<T> *)tw, twlog);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    } else {
        return -2;
    }
}

template <typename T, int N>
static int run_spectra(bool inverse, const void *src, void *dst, int B, int nsrc, int M, int ny, int ldc,
                       const void *tw, int twlog, hipStream_t st)
{
    if constexpr (use_ws<N>()) {
        using C = WsCfg<T, N>;
        constexpr int chunk = 8;
        const long nblk = ((long)(M + 1) * B + C::G - 1) / C::G;
        const long nchunk = (nsrc + chunk - 1) / chunk;
        if (nblk < 1 || nchunk < 1) return 0;
        if (!inverse) {
            const size_t lds = ((size_t)C::G * (2 * C::CW + C::NW * C::XW) + C::TWW) * sizeof(T);
            if (lds > lds_limit()) return -3;
            hipLaunchKernelGGL((col_spectra_ws_kernel<T, N>), dim3((unsigned)nblk, (unsigned)nchunk),
                               dim3(C::THREADS), lds, st, (const cx<T> *)src, (cx<T> *)dst, B, nsrc, M, ny, ldc,
                               chunk, (const cx<T> *)tw, twlog);
        } else {
            const size_t lds = ((size_t)C::G * (2 * N + C::NW * C::XW) + C::TWW) * sizeof(T);
            if (lds > lds_limit()) return -3;
            hipLaunchKernelGGL((col_inverse_ws_kernel<T, N>), dim3((unsigned)nblk, (unsigned)nchunk),
                               dim3(C::THREADS), lds, st, (const cx<T> *)src, (cx<T> *)dst, B, nsrc, M, ny, ldc,
                               chunk, (const cx<T> *)tw, twlog);
        }
        return hipGetLastError() == hipSuccess ? 0 : -1;
    } else {
        return -2;
    }
}

template <typename T, bool ADJ>
static int run_toep(const void *X, const void *spec, void *out, int B, int nz, int nlev, int M, int QP, int Cs, int Ct,
                    unsigned im, unsigned yo, bool accumulate, hipStream_t st)
{
    constexpr int TL = toep_tl<T>(), per = (kToepThreads / 64) * TL;
    const int ntile = (QP + 31) / 32;
    const int nzb = ADJ ? (nz + per - 1) / per : Cs * ((nlev + per - 1) / per);
    const long ntt = (long)ntile * (M + 1);
    const long nblk = ((ntt + 7) / 8) * 8 * nzb;
    const size_t lds = toep_lds_bytes<T, TL>();
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((levels_toeplitz_kernel<T, TL, ADJ>), dim3((unsigned)nblk, (unsigned)B), dim3(kToepThreads),
                       lds, st, (const cx<T> *)X, (const T *)spec, (cx<T> *)out, nz, nlev, M, QP, Cs, Ct, im, yo,
                       ntile, nzb, accumulate ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename TO, int N>
static int run_kgen(const void *Rk, void *spec, int nl, int n0, int Cs, int nz, int M,
                    unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    using C = ColCfg<double, N>;
    const long groups = (long)nl * Cs * (M + 1);
    const long nblk = (groups + C::G - 1) / C::G;
    const size_t lds = (size_t)C::G * 2 * C::FFTK::lds_words() * sizeof(double);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((col_kgen_kernel<TO, N>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                       (const cx<double> *)Rk, (TO *)spec, nl, n0, Cs, nz, M, imag_mask, yodd_mask,
                       (const cx<double> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define GF_COL_SIZES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// The full tensor set gz, gxx, gxy, gxz, gyy, gyz in slot order: gxz and gyz
// have imaginary spectra, gxy and gyz are odd in y.
constexpr unsigned KIND_FULL6_IM = (1u << 3) | (1u << 5);
constexpr unsigned KIND_FULL6_YO = (1u << 2) | (1u << 5);
constexpr int KIND_FULL6 = (int)(KIND_FULL6_IM | (KIND_FULL6_YO << 8));

template <typename T, int N>
static int fwd_c(int Cs, int Ct, const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc,
                 int nsplit, int lps, const NyqSplit &nq, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs == 6 && im == KIND_FULL6_IM && yo == KIND_FULL6_YO)
        return run_fwd<T, N, 6, KIND_FULL6>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs == 1 && im == 0 && yo == 0)
        return run_fwd<T, N, 1, 0>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs <= 1) return run_fwd<T, N, 1, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_fwd<T, N, 3, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    return run_fwd<T, N, 6, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
}

template <typename T, int N>
static int adj_c(int Cs, int Ct, const void *R, const void *spec, void *Gout, int B, int nz, int M, int ny, int ldc,
                 int nsplit, int lps, const NyqSplit &nq, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs == 6 && im == KIND_FULL6_IM && yo == KIND_FULL6_YO)
        return run_adj<T, N, 6, KIND_FULL6>(R, spec, Gout, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs == 1 && im == 0 && yo == 0)
        return run_adj<T, N, 1, 0>(R, spec, Gout, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs <= 1) return run_adj<T, N, 1, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_adj<T, N, 3, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
    return run_adj<T, N, 6, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, Ct, nsplit, lps, nq, im, yo, tw, twlog, st);
}

int launch_col_forward(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz,
                       int M, int ny, int ldc, int Cs, int Ct, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    // the kernels skip the upper half of each column (zero padding)
    if (Cs < 1 || Cs > 6 || Ct < Cs || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? fwd_c<double, NN>(Cs, Ct, R, spec, D, B, nz, M, ny, ldc, nsplit, lps, nq, imag_mask,    \
                                        yodd_mask, tw, twlog, st)                                \
                    : fwd_c<float, NN>(Cs, Ct, R, spec, D, B, nz, M, ny, ldc, nsplit, lps, nq, imag_mask,     \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_adjoint(bool fp64, int py, const void *R, const void *spec, void *Gout, int B,
                       int nz, int M, int ny, int ldc, int Cs, int Ct, int nsplit, int lps, const NyqSplit &nq, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || Cs > 6 || Ct < Cs || ny < 1 || 2 * ny > py || ldc < ny) return -2;   // upper half of columns skipped
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? adj_c<double, NN>(Cs, Ct, R, spec, Gout, B, nz, M, ny, ldc, nsplit, lps, nq, imag_mask, \
                                        yodd_mask, tw, twlog, st)                                \
                    : adj_c<float, NN>(Cs, Ct, R, spec, Gout, B, nz, M, ny, ldc, nsplit, lps, nq, imag_mask,  \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_forward_levels(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz, int M,
                              int ny, int ldc, int Cs, int nlev, int nsplit, int lps, const NyqSplit &nq,
                              unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || nlev < 1 || nlev * Cs > 6 || (nlev + 1) * Cs > 12 || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                             \
    case NN:                                                                                                 \
        return fp64 ? run_levels<double, NN>(R, spec, D, B, nz, M, ny, ldc, Cs, nlev, nsplit, lps, nq, imag_mask, \
                                             yodd_mask, tw, twlog, st)                                       \
                    : run_levels<float, NN>(R, spec, D, B, nz, M, ny, ldc, Cs, nlev, nsplit, lps, nq, imag_mask,  \
                                            yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_adjoint_levels(bool fp64, int py, const void *R, const void *spec, void *Gout, int B, int nz, int M,
                              int ny, int ldc, int Cs, int nlev, int nsplit, int lps, const NyqSplit &nq,
                              unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || nlev < 1 || nlev * Cs > 6 || (nlev + 1) * Cs > 12 || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                                 \
    case NN:                                                                                                     \
        return fp64 ? run_levels_adj<double, NN>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nlev, nsplit, lps, nq,      \
                                                 imag_mask, yodd_mask, tw, twlog, st)                            \
                    : run_levels_adj<float, NN>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nlev, nsplit, lps, nq,       \
                                                imag_mask, yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

template <typename T, int N>
static bool levels_supported_of()
{
    if constexpr (use_ws<N>())
        return WsCfg<T, N>::lds_bytes(6) <= lds_limit();
    else
        return false;
}

bool col_levels_supported(bool fp64, int py)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? levels_supported_of<double, NN>() : levels_supported_of<float, NN>();
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return false;
    }
#undef CASE
}

int launch_col_kgen(bool out_fp64, int py, const void *Rk, void *spec, int nl, int n0, int Cs,
                    int nz, int M, unsigned imag_mask, unsigned yodd_mask, const void *tw, int twlog,
                    hipStream_t st)
{
#define CASE(NN)                                                                                  \
    case NN:                                                                                      \
        return out_fp64 ? run_kgen<double, NN>(Rk, spec, nl, n0, Cs, nz, M, imag_mask, yodd_mask, tw, twlog, \
                                               st)                                                      \
                        : run_kgen<float, NN>(Rk, spec, nl, n0, Cs, nz, M, imag_mask, yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

// resident workgroups of the forward pass (the generic-kind instance stands
// for the specialised ones: same LDS, registers within a few)
template <typename T, int N>
static int capacity_of(int Cs)
{
    int nb = 0;
    hipError_t e;
    if constexpr (use_ws<N>()) {
        using C = WsCfg<T, N>;
        if (Cs <= 1)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_ws_kernel<T, N, 1, -1, false>, C::THREADS,
                                                             C::lds_bytes(1));
        else if (Cs <= 3)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_ws_kernel<T, N, 3, -1, false>, C::THREADS,
                                                             C::lds_bytes(3));
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_ws_kernel<T, N, 6, -1, false>, C::THREADS,
                                                             C::lds_bytes(6));
    } else {
        using C = ColCfg<T, N>;
        if (Cs <= 1)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 1, -1>, C::THREADS,
                                                             C::lds_bytes(1, true));
        else if (Cs <= 3)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 3, -1>, C::THREADS,
                                                             C::lds_bytes(3, true));
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, col_forward_kernel<T, N, 6, -1>, C::THREADS,
                                                             C::lds_bytes(6, true));
    }
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

int spec_row_pitch(bool fp64, int py)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? ColCfg<double, NN>::QP : ColCfg<float, NN>::QP;
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return 0;
    }
#undef CASE
}

template <typename T, int N>
static bool supported_of(int Cs)
{
    const int cmax = Cs <= 1 ? 1 : (Cs <= 3 ? 3 : 6);
    if constexpr (use_ws<N>()) {
        return WsCfg<T, N>::lds_bytes(cmax) <= lds_limit();
    } else {
        using C = ColCfg<T, N>;
        return C::lds_bytes(cmax, true) <= lds_limit() && C::lds_bytes(cmax, false) <= lds_limit();
    }
}

bool col_supported(bool fp64, int py, int Cs)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? supported_of<double, NN>(Cs) : supported_of<float, NN>(Cs);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return false;
    }
#undef CASE
}

bool col_nyquist_apart(int py)
{
#define CASE(NN) \
    case NN:     \
        return use_ws<NN>();
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return false;
    }
#undef CASE
}

int spec_position(bool fp64, int py, int ky)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? (int)spec_pos<double, NN>((unsigned)ky) : (int)spec_pos<float, NN>((unsigned)ky);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return ky;
    }
#undef CASE
}

template <typename T, int N>
static constexpr int groups_of()
{
    if constexpr (use_ws<N>())
        return WsCfg<T, N>::G;
    else
        return ColCfg<T, N>::G;
}

int col_forward_groups(bool fp64, int py)
{
#define CASE(NN) \
    case NN:     \
        return fp64 ? groups_of<double, NN>() : groups_of<float, NN>();
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return 1;
    }
#undef CASE
}

int launch_col_spectra(bool fp64, int py, const void *R, void *X, int B, int nsrc, int M, int ny, int ldc,
                       const void *tw, int twlog, hipStream_t st)
{
    if (B < 1 || nsrc < 0 || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                          \
    case NN:                                                                                              \
        return fp64 ? run_spectra<double, NN>(false, R, X, B, nsrc, M, ny, ldc, tw, twlog, st)           \
                    : run_spectra<float, NN>(false, R, X, B, nsrc, M, ny, ldc, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_inverse(bool fp64, int py, const void *X, void *D, int B, int nsrc, int M, int ny, int ldc,
                       const void *tw, int twlog, hipStream_t st)
{
    if (B < 1 || nsrc < 0 || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                          \
    case NN:                                                                                              \
        return fp64 ? run_spectra<double, NN>(true, X, D, B, nsrc, M, ny, ldc, tw, twlog, st)            \
                    : run_spectra<float, NN>(true, X, D, B, nsrc, M, ny, ldc, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

bool col_spectra_supported(int py)
{
#define CASE(NN) \
    case NN:     \
        return use_ws<NN>();
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return false;
    }
#undef CASE
}

int launch_levels_forward(bool fp64, int py, const void *X, const void *spec, void *Dh, int B, int nz, int nlev, int M,
                          int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, hipStream_t st)
{
    const int QP = spec_row_pitch(fp64, py);
    if (QP <= 0 || B < 1 || nz < 1 || nlev < 1 || Cs < 1 || Cs > kColMaxSpec || Ct < Cs) return -2;
    return fp64 ? run_toep<double, false>(X, spec, Dh, B, nz, nlev, M, QP, Cs, Ct, imag_mask, yodd_mask, false, st)
                : run_toep<float, false>(X, spec, Dh, B, nz, nlev, M, QP, Cs, Ct, imag_mask, yodd_mask, false, st);
}

int launch_levels_adjoint(bool fp64, int py, const void *Rh, const void *spec, void *Gh, int B, int nz, int nlev, int M,
                          int Cs, int Ct, unsigned imag_mask, unsigned yodd_mask, bool accumulate, hipStream_t st)
{
    const int QP = spec_row_pitch(fp64, py);
    if (QP <= 0 || B < 1 || nz < 1 || nlev < 1 || Cs < 1 || Cs > kColMaxSpec || Ct < Cs) return -2;
    return fp64 ? run_toep<double, true>(Rh, spec, Gh, B, nz, nlev, M, QP, Cs, Ct, imag_mask, yodd_mask, accumulate, st)
                : run_toep<float, true>(Rh, spec, Gh, B, nz, nlev, M, QP, Cs, Ct, imag_mask, yodd_mask, accumulate, st);
}

}  // namespace gf
