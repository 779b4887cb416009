// Device building blocks: complex arithmetic, small DFTs and a workgroup
// Stockham FFT whose data live in registers between LDS exchanges.
//
// The FFTs implement the discrete Fourier transforms that diagonalise the
// circulant embedding of each BTTB layer block (section 2.2.3, eq. 18):
// forward X[k] = sum_j x[j] exp(-2 pi i j k / N), inverse with exp(+...),
// both unnormalised.
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T re, T im) { return cx<T>{re, im}; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return cx<T>{a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return cx<T>{a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b)
{
    return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return cx<T>{a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return cx<T>{a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot(cx<T> a)
{
    return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// Workgroup barrier for LDS traffic only: this wave's LDS operations have
// completed, then all waves meet.  Unlike __syncthreads() (a workgroup fence,
// which also waits for every outstanding global load, including asynchronous
// global-to-LDS copies still streaming into another buffer), it leaves global
// loads in flight.  The memory clobber keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int X>
struct ilog2 {
    static constexpr int value = 1 + ilog2<X / 2>::value;
};
template <>
struct ilog2<1> {
    static constexpr int value = 0;
};

// ---------------------------------------------------------------- DFTs ----
template <typename T, int R, bool INV>
struct dft;

template <typename T, bool INV>
struct dft<T, 1, INV> {
    __device__ __forceinline__ static void run(cx<T> *) {}
};

template <typename T, bool INV>
struct dft<T, 2, INV> {
    __device__ __forceinline__ static void run(cx<T> *a)
    {
        cx<T> t = a[0];
        a[0] = add(t, a[1]);
        a[1] = sub(t, a[1]);
    }
};

template <typename T, bool INV>
struct dft<T, 4, INV> {
    __device__ __forceinline__ static void run(cx<T> *a)
    {
        cx<T> t0 = add(a[0], a[2]);
        cx<T> t1 = sub(a[0], a[2]);
        cx<T> t2 = add(a[1], a[3]);
        cx<T> t3 = rot<T, INV>(sub(a[1], a[3]));
        a[0] = add(t0, t2);
        a[2] = sub(t0, t2);
        a[1] = add(t1, t3);
        a[3] = sub(t1, t3);
    }
};

template <typename T, bool INV>
struct dft<T, 8, INV> {
    __device__ __forceinline__ static void run(cx<T> *a)
    {
        const T h = T(0.70710678118654752440084436210484903928);
        cx<T> e[4] = {a[0], a[2], a[4], a[6]};
        cx<T> o[4] = {a[1], a[3], a[5], a[7]};
        dft<T, 4, INV>::run(e);
        dft<T, 4, INV>::run(o);
        // o[k] *= w8^k, w8 = exp(-+ i pi / 4)
        cx<T> o1 = INV ? cx<T>{(o[1].re - o[1].im) * h, (o[1].re + o[1].im) * h}
                       : cx<T>{(o[1].re + o[1].im) * h, (o[1].im - o[1].re) * h};
        cx<T> o2 = rot<T, INV>(o[2]);
        cx<T> o3 = INV ? cx<T>{-(o[3].re + o[3].im) * h, (o[3].re - o[3].im) * h}
                       : cx<T>{(o[3].im - o[3].re) * h, -(o[3].re + o[3].im) * h};
        a[0] = add(e[0], o[0]);
        a[4] = sub(e[0], o[0]);
        a[1] = add(e[1], o1);
        a[5] = sub(e[1], o1);
        a[2] = add(e[2], o2);
        a[6] = sub(e[2], o2);
        a[3] = add(e[3], o3);
        a[7] = sub(e[3], o3);
    }
};

// ------------------------------------------------------------ twiddles ----
// tw[m] = exp(-2 pi i m / TL) for m in [0, TL), TL = 2^twlog (a power of two
// no smaller than any transform length in use).  W(a, L) = exp(-+2 pi i a / L).
//
// The table pointer is passed through an empty asm statement at every stage:
// the compiler then cannot hoist twiddle loads out of the stage (or out of a
// loop that repeats the transform), which would keep dozens of values live
// in registers for the whole kernel.
template <typename T>
__device__ __forceinline__ const cx<T> *opaque(const cx<T> *p)
{
    asm volatile("" : "+s"(p));
    return p;
}

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T> *__restrict__ tw, int twlog, unsigned a, int logL)
{
    cx<T> w = tw[a << (unsigned)(twlog - logL)];
    return INV ? conjg(w) : w;
}

// ------------------------------------------------------ workgroup FFT ----
// One length-N transform per group of NT threads; PPT = N/NT points per
// thread.  Stockham autosort: stage s with radix R and span Ns combines
// elements j + k N/R (k < R) of butterfly j after twiddling by
// W((j mod Ns) k, Ns R) and writes them to (j div Ns) Ns R + (j mod Ns) + k Ns.
// Register slot v[m R + k] of thread t holds element t + NT (m + k PPT/R);
// with R = PPT this is element t + NT k.  The same layout holds on output
// (with the radix of the last stage), so callers index slots through
// elem_in()/elem_out().
//
// LDS per group: with XSPLIT = false, two arrays (re, im) of lds_words()
// entries; with XSPLIT = true one array, through which the real and the
// imaginary parts are exchanged one after the other (half the LDS, twice the
// barriers).  Exchange indices are padded per stage (see xpad) to avoid bank
// conflicts.
// With WAVESYNC (a group within one wave: NT dividing 64, groups aligned to
// waves) the exchanges are ordered by waiting for this wave's own LDS
// operations instead of a workgroup barrier.
template <typename T, int N, int NT, int R, bool XSPLIT = false, bool TWS = false, bool WAVESYNC = false>
struct BlockFFT {
    static_assert(!WAVESYNC || (NT <= 64 && 64 % NT == 0), "wave-local exchange needs transforms within one wave");
    __device__ __forceinline__ static void xsync()
    {
        if constexpr (WAVESYNC)
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        else
            lds_barrier();
    }
    static constexpr int PPT = N / NT;
    static constexpr int LOGN = ilog2<N>::value;
    static constexpr int LOGR = ilog2<R>::value;
    static_assert(N % NT == 0, "N must be a multiple of NT");
    static_assert(PPT % R == 0, "PPT must be a multiple of R");
    static constexpr int LAST_R = (LOGN % LOGR == 0) ? R : (1 << (LOGN % LOGR));
    static constexpr int NSTAGES = (LOGN + LOGR - 1) / LOGR;

    // LDS layout of the exchange that follows a stage of span Ns and radix
    // RS.  The stage writes element base + k Ns (k < RS) and the next stage
    // reads consecutive elements.  A padding of c words every 2^P elements
    // keeps both access patterns free of LDS bank conflicts (64 banks of 4
    // bytes, 256 bytes a cycle): after span 1 (a stride of RS elements across
    // lanes) one word every 256 bytes; after spans 1 < Ns < 64 (runs of Ns
    // lanes) Ns words every butterfly group of Ns RS elements; spans of 64
    // and more write whole rows and need none.  The padding is additive, so
    // constant offsets still fold into the instructions' immediates.
    static constexpr int LOGE = ilog2<256 / sizeof(T)>::value;  // elements a bank row
    __host__ __device__ static constexpr int xpad_words(int ns) { return ns == 1 ? 1 : (ns >= 64 ? 0 : ns); }
    __host__ __device__ static constexpr int xpad_shift(int ns, int rs)
    {
        int p = 0;
        for (int x = ns * rs; x > 1; x >>= 1) ++p;
        return ns == 1 ? LOGE : p;
    }
    template <int Ns, int RS>
    __device__ __forceinline__ static unsigned xpad(unsigned i)
    {
        constexpr int c = xpad_words(Ns), p = xpad_shift(Ns, RS);
        if constexpr (c == 0)
            return i;
        else
            return i + c * (i >> p);
    }
    // T words of one exchange array: the largest padded index of any exchange
    __host__ __device__ static constexpr int lds_words()
    {
        int w = N;
        int ns = 1, rs = (N >= R ? R : N);
        while (ns * rs < N) {
            const int e = N + xpad_words(ns) * ((N - 1) >> xpad_shift(ns, rs));
            if (e > w) w = e;
            ns *= rs;
            rs = (ns * R <= N) ? R : N / ns;
        }
        return w;
    }
    // T words of LDS one group needs
    __host__ __device__ static constexpr int lds_group_words() { return (XSPLIT ? 1 : 2) * lds_words(); }
    // layout of data handed to or taken from the transform through LDS by
    // callers: element i at word i
    __device__ __forceinline__ static unsigned pad(unsigned i) { return i; }

    // element index (multiplier of NT plus t) held by register slot s, for a
    // stage of radix RR
    __host__ __device__ static constexpr int slot_elem(int s, int RR)
    {
        return (s / RR) + (s % RR) * (PPT / RR);
    }
    __host__ __device__ static constexpr int first_r() { return N >= R ? R : N; }
    // element multiplier of slot s on input / output
    __host__ __device__ static constexpr int elem_in(int s) { return slot_elem(s, first_r()); }
    __host__ __device__ static constexpr int elem_out(int s) { return slot_elem(s, LAST_R); }

    // Per-stage twiddle table (TWS): for every stage of span Ns > 1 the Ns
    // values W(jm, Ns RS), jm < Ns, stored one stage after the other, real
    // parts then imaginary parts.  Lanes of a stage read consecutive entries
    // (no LDS bank conflicts); the other powers are formed by products.
    __host__ __device__ static constexpr int stage_radix(int Ns) { return (Ns * R <= N) ? R : N / Ns; }
    __host__ __device__ static constexpr int stw_offset(int Ns)
    {
        int off = 0;
        for (int s = R; s < Ns; s *= R) off += s;
        return off;
    }
    __host__ __device__ static constexpr int stw_entries() { return stw_offset(N); }

    // Fill the per-stage table (tre: stw_entries() real parts, then as many
    // imaginary parts) from the global table of length 2^twlog.
    __device__ static void load_stage_table(T *tre, const cx<T> *__restrict__ tw, int twlog, unsigned tid,
                                            unsigned nthreads)
    {
        T *tim = tre + stw_entries();
        for (unsigned i = tid; i < (unsigned)stw_entries(); i += nthreads) {
            unsigned ns = R, off = 0;
            while (i >= off + ns) {
                off += ns;
                ns *= R;
            }
            const unsigned len = ns * (unsigned)stage_radix((int)ns);
            const cx<T> w = tw[(i - off) << (unsigned)(twlog - __builtin_ctz(len))];
            tre[i] = w.re;
            tim[i] = w.im;
        }
    }

    // With TWS, tw points to the per-stage table in LDS (twlog unused).
    template <int Ns, bool INV>
    __device__ __forceinline__ static void stage(cx<T> (&v)[PPT], T *sre, T *sim, unsigned t,
                                                 const cx<T> *__restrict__ tw, int twlog)
    {
        constexpr int RS = (Ns * R <= N) ? R : (N / Ns);
        constexpr int NB = PPT / RS;
        constexpr int LOGL = ilog2<Ns * RS>::value;
        const cx<T> *tws = TWS ? tw : opaque(tw);
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const unsigned j = t + m * NT;
            const unsigned jm = j & (Ns - 1);
            if (Ns > 1) {
                cx<T> w[RS > 1 ? RS : 2];
                if constexpr (TWS) {
                    const T *tre = reinterpret_cast<const T *>(tws);
                    constexpr int off = stw_offset(Ns);
                    w[1] = cx<T>{tre[off + jm], tre[stw_entries() + off + jm]};
                    if (INV) w[1] = conjg(w[1]);
                    if constexpr (RS > 2) w[2] = mul(w[1], w[1]);
                    if constexpr (RS > 4) w[4] = mul(w[2], w[2]);
                } else {
                    // fetch w^1, w^2, w^4 and form the other powers by at
                    // most two products (3 table reads per butterfly instead
                    // of RS-1)
                    w[1] = twiddle<T, INV>(tws, twlog, jm, LOGL);
                    if constexpr (RS > 2) w[2] = twiddle<T, INV>(tws, twlog, jm * 2, LOGL);
                    if constexpr (RS > 4) w[4] = twiddle<T, INV>(tws, twlog, jm * 4, LOGL);
                }
                if constexpr (RS > 3) w[3] = mul(w[1], w[2]);
                if constexpr (RS > 4) {
                    w[5] = mul(w[1], w[4]);
                    w[6] = mul(w[2], w[4]);
                    w[7] = mul(w[3], w[4]);
                }
#pragma unroll
                for (int k = 1; k < RS; ++k) v[m * RS + k] = mul(v[m * RS + k], w[k]);
            }
            dft<T, RS, INV>::run(&v[m * RS]);
        }
        if constexpr (Ns * RS < N) {
            constexpr int NS2 = Ns * RS;
            constexpr int R2 = (NS2 * R <= N) ? R : (N / NS2);
            constexpr int NB2 = PPT / R2;
#pragma unroll
            for (int part = 0; part < (XSPLIT ? 2 : 1); ++part) {
                xsync();
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const unsigned j = t + m * NT;
                    const unsigned jm = j & (Ns - 1);
                    const unsigned base = (j >> ilog2<Ns>::value) * Ns * RS + jm;
#pragma unroll
                    for (int k = 0; k < RS; ++k) {
                        const unsigned idx = xpad<Ns, RS>(base + k * Ns);
                        if (XSPLIT) {
                            sre[idx] = part == 0 ? v[m * RS + k].re : v[m * RS + k].im;
                        } else {
                            sre[idx] = v[m * RS + k].re;
                            sim[idx] = v[m * RS + k].im;
                        }
                    }
                }
                xsync();
                // every value of this part has been written; read the next
                // stage's inputs (slot order m*R2 + k)
#pragma unroll
                for (int m = 0; m < NB2; ++m)
#pragma unroll
                    for (int k = 0; k < R2; ++k) {
                        const unsigned idx = xpad<Ns, RS>(t + m * NT + k * (N / R2));
                        if (XSPLIT) {
                            // part 0 replaces only the real fields and part 1
                            // only the imaginary ones, so the imaginary parts
                            // written in part 1 are still this stage's
                            if (part == 0)
                                v[m * R2 + k].re = sre[idx];
                            else
                                v[m * R2 + k].im = sre[idx];
                        } else {
                            v[m * R2 + k] = cx<T>{sre[idx], sim[idx]};
                        }
                    }
            }
            stage<NS2, INV>(v, sre, sim, t, tw, twlog);
        }
    }

    // Transform in place.  All threads of the workgroup must call it (it
    // contains workgroup barriers); sre/sim point to this group's LDS area
    // (sim unused with XSPLIT).
    template <bool INV>
    __device__ __forceinline__ static void run(cx<T> (&v)[PPT], T *sre, T *sim, unsigned t,
                                               const cx<T> *__restrict__ tw, int twlog)
    {
        stage<1, INV>(v, sre, sim, t, tw, twlog);
    }
};

}  // namespace gf
