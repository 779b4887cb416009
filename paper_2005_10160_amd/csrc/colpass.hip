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
    static constexpr int PPT = 8;
    static constexpr int NT = N / PPT;
    static constexpr int RADIX = 8;
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
    // register target: FP32 workgroups fit two per CU by LDS, so ask for two
    // waves per SIMD (at most 256 registers a lane); FP64 ones fit one.
    static constexpr int WAVES_PER_EU = sizeof(T) == 4 ? (THREADS <= 256 ? 2 : 1) : 1;
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
                       cx<T> *__restrict__ D, int B, int nz, int M, int ny, int ldc, int Cs, int lps,
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
                store_column<T, PPT, F, NT>(D + ((((size_t)split * B + w.b) * Cs + c) * M + w.u) * (size_t)ldc,
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
                       cx<T> *__restrict__ Gout, int B, int nz, int M, int ny, int ldc, int Cs, int lps,
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
            const cx<T> *col = column(R, (size_t)w.b * Cs + c, M, w.u, ldc);
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
            if (ky <= N / 2) dst[ky] = (yo && ky == N / 2) ? TO(0) : (TO)(im ? v[s].im : v[s].re);
        }
        // zero the row padding so staged blocks hold no stale values
        if (t < QPO - (N / 2 + 1)) dst[N / 2 + 1 + t] = TO(0);
    }
}

template <typename T, int N, int CMAX, int KIND>
static int run_fwd(const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc, int Cs,
                   int nsplit, int lps, unsigned imag_mask, unsigned yodd_mask, const void *tw,
                   int twlog, hipStream_t st)
{
    using C = ColCfg<T, N>;
    const long groups = (long)(M + 1) * B;
    const long nblk = (groups + C::G - 1) / C::G;
    const size_t lds = C::lds_bytes(CMAX, true);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((col_forward_kernel<T, N, CMAX, KIND>), dim3((unsigned)nblk, (unsigned)nsplit),
                       dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec, (cx<T> *)D,
                       B, nz, M, ny, ldc, Cs, lps, imag_mask, yodd_mask, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int N, int CMAX, int KIND>
static int run_adj(const void *R, const void *spec, void *Gout, int B, int nz, int M, int ny, int ldc, int Cs,
                   int nsplit, int lps, unsigned imag_mask, unsigned yodd_mask, const void *tw,
                   int twlog, hipStream_t st)
{
    using C = ColCfg<T, N>;
    const long groups = (long)(M + 1) * B;
    const long nblk = (groups + C::G - 1) / C::G;
    const size_t lds = C::lds_bytes(CMAX, false);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((col_adjoint_kernel<T, N, CMAX, KIND>), dim3((unsigned)nblk, (unsigned)nsplit),
                       dim3(C::THREADS), lds, st, (const cx<T> *)R, (const T *)spec,
                       (cx<T> *)Gout, B, nz, M, ny, ldc, Cs, lps, imag_mask, yodd_mask,
                       (const cx<T> *)tw, twlog);
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
static int fwd_c(int Cs, const void *R, const void *spec, void *D, int B, int nz, int M, int ny, int ldc,
                 int nsplit, int lps, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs == 6 && im == KIND_FULL6_IM && yo == KIND_FULL6_YO)
        return run_fwd<T, N, 6, KIND_FULL6>(R, spec, D, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs == 1 && im == 0 && yo == 0)
        return run_fwd<T, N, 1, 0>(R, spec, D, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 1) return run_fwd<T, N, 1, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_fwd<T, N, 3, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    return run_fwd<T, N, 6, -1>(R, spec, D, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
}

template <typename T, int N>
static int adj_c(int Cs, const void *R, const void *spec, void *Gout, int B, int nz, int M, int ny, int ldc,
                 int nsplit, int lps, unsigned im, unsigned yo, const void *tw, int twlog,
                 hipStream_t st)
{
    if (Cs == 6 && im == KIND_FULL6_IM && yo == KIND_FULL6_YO)
        return run_adj<T, N, 6, KIND_FULL6>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs == 1 && im == 0 && yo == 0)
        return run_adj<T, N, 1, 0>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 1) return run_adj<T, N, 1, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    if (Cs <= 3) return run_adj<T, N, 3, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
    return run_adj<T, N, 6, -1>(R, spec, Gout, B, nz, M, ny, ldc, Cs, nsplit, lps, im, yo, tw, twlog, st);
}

int launch_col_forward(bool fp64, int py, const void *R, const void *spec, void *D, int B, int nz,
                       int M, int ny, int ldc, int Cs, int nsplit, int lps, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    // the kernels skip the upper half of each column (zero padding)
    if (Cs < 1 || Cs > 6 || ny < 1 || 2 * ny > py || ldc < ny) return -2;
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? fwd_c<double, NN>(Cs, R, spec, D, B, nz, M, ny, ldc, nsplit, lps, imag_mask,    \
                                        yodd_mask, tw, twlog, st)                                \
                    : fwd_c<float, NN>(Cs, R, spec, D, B, nz, M, ny, ldc, nsplit, lps, imag_mask,     \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_col_adjoint(bool fp64, int py, const void *R, const void *spec, void *Gout, int B,
                       int nz, int M, int ny, int ldc, int Cs, int nsplit, int lps, unsigned imag_mask,
                       unsigned yodd_mask, const void *tw, int twlog, hipStream_t st)
{
    if (Cs < 1 || Cs > 6 || ny < 1 || 2 * ny > py || ldc < ny) return -2;   // upper half of columns skipped
#define CASE(NN)                                                                                 \
    case NN:                                                                                     \
        return fp64 ? adj_c<double, NN>(Cs, R, spec, Gout, B, nz, M, ny, ldc, nsplit, lps, imag_mask, \
                                        yodd_mask, tw, twlog, st)                                \
                    : adj_c<float, NN>(Cs, R, spec, Gout, B, nz, M, ny, ldc, nsplit, lps, imag_mask,  \
                                       yodd_mask, tw, twlog, st);
    switch (py) {
        GF_COL_SIZES(CASE)
    default:
        return -2;
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
    using C = ColCfg<T, N>;
    const int cmax = Cs <= 1 ? 1 : (Cs <= 3 ? 3 : 6);
    return C::lds_bytes(cmax, true) <= lds_limit() && C::lds_bytes(cmax, false) <= lds_limit();
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
