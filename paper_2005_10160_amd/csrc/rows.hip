// Row (x-direction) transforms of the 2-D FFT of section 2.2.3 (eq. 18).
//
// Forward: each real row of length Px (only its first `lin` entries are
// nonzero: the zero padding of the circulant embedding) is transformed as a
// half-length complex FFT of z[j] = x[2j] + i x[2j+1], then unpacked to the
// Px/2+1 non-redundant bins X[u].  Bins 0 and Px/2 are real and share unit 0
// (X[0] as its real part, X[Px/2] as its imaginary part), so a row becomes
// M = Px/2 complex units.  Output is written transposed, out[slab][u][y], so
// that the column pass reads each column contiguously; the transposition
// goes through LDS, and consecutive lanes write consecutive rows of one unit.
//
// Inverse: the mirror image: a tile of rows is gathered transposed from
// D[..][u][y], packed back to a half-length complex spectrum, inverse
// transformed, cropped to the first nx outputs (the crop of eq. 18) and
// scaled.
#include "gf_fft.h"
#include "gf_launch.h"

namespace gf {

// The combination that feeds (forward) or reads (inverse) sub-row o: up to
// two sources with weights.  The selection runs over static indices, so the
// combination table stays in scalar registers instead of being fetched from
// memory per lane.
template <typename T>
struct Term {
    int n, s0, s1;
    T w0, w1;
};

template <typename T>
__device__ __forceinline__ Term<T> combo_term(const RowCombo &cmb, int o)
{
    Term<T> r{1, o, o, T(1), T(0)};
    if (cmb.identity) return r;
#pragma unroll
    for (int k = 0; k < kMaxOut; ++k)
        if (o == k) {
            r.n = cmb.nterm[k];
            r.s0 = cmb.src[k][0];
            r.s1 = cmb.nterm[k] > 1 ? cmb.src[k][1] : cmb.src[k][0];
            r.w0 = cmb.nterm[k] > 0 ? (T)cmb.w[k][0] : T(0);
            r.w1 = cmb.nterm[k] > 1 ? (T)cmb.w[k][1] : T(0);
        }
    return r;
}

// Forward rows (a row of Px = 2M points is a transform of M complex points;
// "points a lane" counts those): 16 points a lane for long rows, real and
// imaginary parts exchanged one after the other through one LDS array per
// row.  Rows per workgroup: within 40 KB of LDS and 512 threads, so that two
// workgroups share a CU and one's loads and stores overlap the other's
// transforms.
// FP32 rows of 1024 points also take 16 points a lane: half a wave per row
// gives sixteen rows a workgroup, whose transposed stores then cover whole
// 128-byte lines (8-byte units of 16 consecutive rows; batched 512 x 512 x
// 128 FP32 row pass 3.07-3.12 -> 2.90 ms).
template <typename T, int M>
struct RowCfgF {
    static constexpr int PPT = (M >= 1024 || (M == 512 && sizeof(T) == 4)) ? 16 : ((M >= 8) ? 8 : M);
    static constexpr int NT = M / PPT;
    static constexpr int RADIX = PPT >= 8 ? 8 : PPT;
    // stage twiddles from a per-stage table in LDS, filled once per
    // workgroup (global table lookups, with their index and address
    // arithmetic per butterfly, cost FP64 0.62 -> 0.57 ms and FP32
    // 0.37 -> 0.33 ms at 1024 x 1024 x 100)
    static constexpr bool TWS = true;
    // a row's lanes lie within one wave: its exchanges need only the wave's
    // own LDS ordering
    using FFT = BlockFFT<T, M, NT, RADIX, true, TWS, (64 % NT) == 0>;
    static constexpr int TWW = TWS ? ((2 * FFT::stw_entries() + 16 / (int)sizeof(T) - 1) / (16 / (int)sizeof(T))) * (16 / (int)sizeof(T)) : 0;
    static constexpr int W = FFT::lds_words();
    static constexpr int E = 256 / (int)sizeof(T);   // elements of one 256-byte bank row
    static constexpr int tr_with(int kb, int threads)
    {
        int tr = 64;
        while (tr > 1 && (tr * (W + E) * (int)sizeof(T) > kb * 1024 || tr * NT > threads)) tr /= 2;
        return tr;
    }
    // Rows of length 4096 (M = 2048) take two waves each; there rows within
    // 80 KB (one workgroup per CU) double the FP64 row group to four rows,
    // whose transposed stores then cover 64-byte segments instead of 32
    // (FP64 row pass 4.5 -> 3.2 ms at 2048 x 2048 x 100; FP32, already at
    // four rows by the thread limit, was slower with eight).
    static constexpr int TR0 = tr_with(40, 512);
    static constexpr int TR = M >= 2048 ? tr_with(80, 512) : TR0;
    static constexpr int THREADS = TR * NT;
    // row stride = SHIFT mod lc elements, where one LDS cycle serves lc =
    // 128 / sizeof(T) lanes (32 lanes of 4 bytes, 16 of 8) and SHIFT = lc /
    // TR, at least 16 bytes (aligned rows): the lanes of one cycle of the
    // transposed reads, TR rows x SHIFT units, then fall in distinct banks
    static constexpr int LC = 128 / (int)sizeof(T);
    static constexpr int SHIFT = LC / TR > 16 / (int)sizeof(T) ? LC / TR : 16 / (int)sizeof(T);
    static constexpr int WS = W + ((SHIFT - W % LC) % LC + LC) % LC;
    static constexpr int ROW_BYTES = WS * (int)sizeof(T);
    // register target: waves per SIMD for two resident workgroups (one for
    // the larger row groups)
    static constexpr int BPC = TR == TR0 ? 2 : 1;
    static constexpr int WAVES_PER_EU =
        (BPC * THREADS / 256) < 1 ? 1 : ((BPC * THREADS / 256) > 8 ? 8 : BPC * THREADS / 256);
    static constexpr int LDS_BYTES = TR * ROW_BYTES + TWW * (int)sizeof(T);
    static_assert(THREADS == TR * NT && THREADS <= 1024, "a row group is TR rows of NT lanes");
    static_assert(LDS_BYTES <= (TR == TR0 ? 40 : 80) * 1024 + TWW * (int)sizeof(T) && BPC * LDS_BYTES <= 160 * 1024,
                  "the row groups' LDS fits the workgroups per CU the register target assumes");
    static_assert(WS % LC == SHIFT % LC && ROW_BYTES % 16 == 0, "row stride: bank shift, 16-byte aligned rows");
};

// Blocks in XCD-contiguous order: the hardware deals consecutive blocks to
// the eight XCDs in turn, while neighbouring row groups share the 128-byte
// lines of the transposed layout; giving each XCD a contiguous range keeps
// those shared lines in one L2.
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned nb = gridDim.x, xcd = blockIdx.x % 8u, k = blockIdx.x / 8u;
    const unsigned q = nb / 8u, rem = nb % 8u;
    return xcd * q + min(xcd, rem) + k;
}

// Inverse rows: full complex exchange; 8 points a lane, 16 for FP32 rows of
// 1024 points and more: half as many lanes a row gives twice the rows a
// workgroup, so that the transposed gather reads runs of twice the length
// (FP32 inverse rows at 1024^2 x 100 0.44 -> 0.33 ms, 100 levels 2.67 ->
// 2.00 ms, batched 512^2 x 128 3.37 -> 2.96 ms).
template <typename T, int M>
struct RowCfg {
    static constexpr int PPT = (M >= 512 && sizeof(T) == 4) ? 16 : ((M >= 8) ? 8 : M);
    static constexpr int NT = M / PPT;
    static constexpr int RADIX = PPT >= 8 ? 8 : PPT;
    // FP32: stage twiddles from a per-stage table in LDS (batched inverse
    // rows at 512 x 512 x 128 4.18 -> 3.81 ms); in FP64 the table's LDS
    // leaves fewer workgroups per CU (100-level inverse rows 3.9 -> 5.7 ms)
    static constexpr bool TWS = sizeof(T) == 4;
    using FFT = BlockFFT<T, M, NT, RADIX, false, TWS>;
    // stage twiddle table after the rows (TWS)
    static constexpr int TWW = TWS ? 2 * FFT::stw_entries() : 0;
    // one word beyond the transform's arrays: element M holds the packed
    // Nyquist bin X[M] before the half-length spectrum is formed
    static constexpr int W = FFT::lds_words() + 1;
    // row stride (re and im arrays) for a group of tr rows: S mod lc
    // elements, where one LDS cycle serves lc = 128 / sizeof(T) lanes (32
    // lanes of 4 bytes, 16 of 8) and S = lc / tr, at least 16 bytes (aligned
    // rows): the lanes of one cycle of the transposed gather, tr rows x S
    // units, then fall in distinct banks
    static constexpr int stride_for(int tr)
    {
        const int lc = 128 / (int)sizeof(T), al = 16 / (int)sizeof(T);
        const int sh = lc / tr > al ? lc / tr : al;
        return 2 * W + ((lc + sh - (2 * W) % lc) % lc);
    }
    // rows per workgroup: a power of two within 80 KB of LDS (two workgroups
    // per CU) and 1024 threads, 512 in FP32 (two workgroups then share a CU
    // where registers leave room for one of 1024 threads: batched 512 x 512
    // x 128 inverse rows 3.9 -> 3.4 ms, 100-level inverse rows 2.9 -> 2.6 ms)
    static constexpr int MAXT = sizeof(T) == 4 ? 512 : 1024;
    static constexpr int tr_calc()
    {
        int tr = 64;
        while (tr > 1 && (tr * stride_for(tr) * (int)sizeof(T) > 80 * 1024 || tr * NT > MAXT)) tr /= 2;
        return tr;
    }
    static constexpr int TR = tr_calc();
    static constexpr int THREADS = TR * NT;
    static constexpr int RWS = stride_for(TR);
    static constexpr int ROW_BYTES = RWS * (int)sizeof(T);
    // register target: two resident workgroups (512-thread FP64 workgroups
    // need at most 128 registers a lane); larger workgroups fit one
    static constexpr int WAVES_PER_EU = THREADS <= 512 ? 2 * THREADS / 256 : 1;
    static constexpr int LDS_BYTES = TR * ROW_BYTES + TWW * (int)sizeof(T);
    static_assert(THREADS == TR * NT && THREADS <= 1024, "a row group is TR rows of NT lanes");
    static_assert(THREADS > 512 || 2 * LDS_BYTES <= 160 * 1024,
                  "two workgroups of at most 512 threads share a CU's LDS");
    static_assert(RWS % (128 / (int)sizeof(T)) ==
                      ((128 / (int)sizeof(T)) / TR > 16 / (int)sizeof(T) ? (128 / (int)sizeof(T)) / TR
                                                                       : 16 / (int)sizeof(T)) % (128 / (int)sizeof(T)) &&
                      ROW_BYTES % 16 == 0,
                  "row stride: bank shift, 16-byte aligned rows");
};

template <typename T, int M, bool HALF>
__global__ void __launch_bounds__((RowCfgF<T, M>::THREADS))
    __attribute__((amdgpu_waves_per_eu(RowCfgF<T, M>::WAVES_PER_EU)))
    row_r2c_kernel(const T *__restrict__ in, long row_len, int lin, int rows, int ldc, int nsub, int src_per_b,
                   long nrows_total, RowCombo cmb, cx<T> *__restrict__ out, long out_bslabs,
                   const cx<T> *__restrict__ tw, int twlog)
{
    using C = RowCfgF<T, M>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, TR = C::TR, W = C::WS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    const long gr0 = (long)xcd_block() * TR;
    const long gr = gr0 + g;
    const cx<T> *ftw = tw;
    if constexpr (C::TWS) {
        F::load_stage_table(lds, tw, twlog, threadIdx.x, C::THREADS);
        ftw = reinterpret_cast<const cx<T> *>(lds);
        lds += C::TWW;
    }
    T *sre = lds + (size_t)g * W;

    // Loads and the transform.  With HALF (lin <= M: a row whose nonzero
    // samples lie in its first half, the zero padding of the circulant
    // embedding) the packed inputs of the upper half of the half-length
    // transform are zero: they are taken as literal zeros (no loads) and the
    // first stage folds them away.
    cx<T> v[PPT];
    if (gr < nrows_total) {
        const long per_b = (long)nsub * rows;
        const int b = (int)(gr / per_b);
        const int s = (int)((gr / rows) % nsub);
        const int y = (int)(gr % rows);
        const Term<T> tm = combo_term<T>(cmb, s);
        const int nterm = tm.n, src0 = tm.s0, src1 = tm.s1;
        const T w0 = tm.w0, w1 = tm.w1;
        const T *r0 = in + (((long)b * src_per_b + src0) * rows + y) * row_len;
        const T *r1 = in + (((long)b * src_per_b + src1) * rows + y) * row_len;
        // Loads are unconditional (indices clamped into the row, values
        // selected afterwards): a guarded load would wait for its data at the
        // branch join and serialise the row.
        const bool pairs = nterm == 1 && ((row_len | lin) & 1) == 0 &&
                           ((reinterpret_cast<size_t>(in) & (2 * sizeof(T) - 1)) == 0);
        if (pairs) {  // (x[2j], x[2j+1]) as one vector
            cx<T> pr[PPT];
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                if (HALF && F::elem_in(sl) >= PPT / 2) continue;
                const unsigned j = t + NT * F::elem_in(sl);
                pr[sl] = *reinterpret_cast<const cx<T> *>(r0 + 2 * (2 * j < (unsigned)lin ? j : 0u));
            }
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_in(sl);
                v[sl] = (HALF && F::elem_in(sl) >= PPT / 2) || 2 * j >= (unsigned)lin
                            ? cx<T>{T(0), T(0)}
                            : cx<T>{w0 * pr[sl].re, w0 * pr[sl].im};
            }
        } else {
            T e0[PPT], o0[PPT];
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_in(sl);
                const unsigned x0 = 2 * j, x1 = 2 * j + 1;
                e0[sl] = r0[x0 < (unsigned)lin ? x0 : 0u];
                o0[sl] = r0[x1 < (unsigned)lin ? x1 : 0u];
            }
            if (nterm > 1) {
                T e1[PPT], o1[PPT];
#pragma unroll
                for (int sl = 0; sl < PPT; ++sl) {
                    const unsigned j = t + NT * F::elem_in(sl);
                    const unsigned x0 = 2 * j, x1 = 2 * j + 1;
                    e1[sl] = r1[x0 < (unsigned)lin ? x0 : 0u];
                    o1[sl] = r1[x1 < (unsigned)lin ? x1 : 0u];
                }
#pragma unroll
                for (int sl = 0; sl < PPT; ++sl) {
                    e0[sl] = w0 * e0[sl] + w1 * e1[sl];
                    o0[sl] = w0 * o0[sl] + w1 * o1[sl];
                }
            } else {
#pragma unroll
                for (int sl = 0; sl < PPT; ++sl) {
                    e0[sl] *= w0;
                    o0[sl] *= w0;
                }
            }
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_in(sl);
                v[sl] = (HALF && F::elem_in(sl) >= PPT / 2)
                            ? cx<T>{T(0), T(0)}
                            : cx<T>{2 * j < (unsigned)lin ? e0[sl] : T(0), 2 * j + 1 < (unsigned)lin ? o0[sl] : T(0)};
            }
        }
    } else {
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) v[sl] = cx<T>{T(0), T(0)};
    }

    if constexpr (C::TWS) __syncthreads();   // the stage table is in place
    F::template run<false>(v, sre, nullptr, t, ftw, twlog);

    // Unpack X[u] = Xe[u] + w^u Xo[u] (w = exp(-2 pi i / Px)) in a row-fastest
    // mapping and store transposed.  Item i of this thread is row r = it % TR,
    // unit u = it / TR with it = threadIdx.x + i * THREADS (M * TR = PPT *
    // THREADS items).  Z[u] and Z[M-u] pass through LDS in two halves.
    T are[PPT], bre[PPT], aim[PPT], bim[PPT];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        __syncthreads();
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) sre[F::pad(t + NT * F::elem_out(sl))] = part == 0 ? v[sl].re : v[sl].im;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const unsigned it = threadIdx.x + i * C::THREADS;
            const unsigned r = it % TR, u = it / TR;
            const T *q = lds + (size_t)r * W;
            const T a = q[F::pad(u)], bb = q[F::pad((M - u) & (M - 1))];
            if (part == 0) {
                are[i] = a;
                bre[i] = bb;
            } else {
                aim[i] = a;
                bim[i] = bb;
            }
        }
    }
    const int logpx = ilog2<2 * M>::value;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const unsigned it = threadIdx.x + i * C::THREADS;
        const unsigned r = it % TR, u = it / TR;
        const long grr = gr0 + r;
        if (grr >= nrows_total) continue;
        cx<T> X;
        if (u == 0) {  // X[0] = Re Z0 + Im Z0, X[M] = Re Z0 - Im Z0, both real
            X = cx<T>{are[i] + aim[i], are[i] - aim[i]};
        } else {
            const cx<T> zk{are[i], aim[i]};
            const cx<T> zm{bre[i], -bim[i]};   // conj(Z[M-u])
            const cx<T> xe = scale(add(zk, zm), T(0.5));
            const cx<T> dd = sub(zk, zm);
            const cx<T> xo{dd.im * T(0.5), -dd.re * T(0.5)};  // (zk - conj zm) / (2i)
            const cx<T> w = twiddle<T, false>(tw, twlog, u, logpx);
            X = add(xe, mul(w, xo));
        }
        const long slab = grr / rows;   // b * nsub + s, written to slab b * out_bslabs + s
        const long oslab = (slab / nsub) * out_bslabs + slab % nsub;
        const int y = (int)(grr % rows);
        out[(oslab * M + u) * (long)ldc + y] = X;
    }
}

template <typename T, int M>
__global__ void __launch_bounds__((RowCfg<T, M>::THREADS))
    __attribute__((amdgpu_waves_per_eu(RowCfg<T, M>::WAVES_PER_EU)))
    row_c2r_kernel(const cx<T> *__restrict__ D, long split_stride, int nsplit, int nsrc, int rows, int ldc,
                   int nsub, long nrows_total, RowCombo cmb, const T *__restrict__ Dny, int nchunk,
                   int nbatch, T *__restrict__ out, long out_bstride, int accumulate, int nx_out, T sc,
                   const cx<T> *__restrict__ tw, int twlog)
{
    using C = RowCfg<T, M>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, TR = C::TR, W = C::W;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const long gr0 = (long)xcd_block() * TR;   // XCD-contiguous row groups

    // gather X(row)[u] transposed (consecutive lanes read consecutive rows),
    // summing the per-split partials.  Thread item i covers row
    // threadIdx.x % TR (the same for every item, as THREADS = TR * NT) and
    // unit threadIdx.x / TR + i * NT.
    bool two = false;   // some output combines two spectra (gzz)
    if (!cmb.identity)
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o) two |= o < nsub && cmb.nterm[o] > 1;
    const unsigned r0 = threadIdx.x % TR, u0 = threadIdx.x / TR;
    long off0, off1;
    T wa, wb;
    {
        const long grr = gr0 + r0;
        const bool valid = grr < nrows_total;
        const long gc = valid ? grr : 0;
        const long per_b = (long)nsub * rows;
        const int b = (int)(gc / per_b);
        const int o = (int)((gc / rows) % nsub);
        const int y = (int)(gc % rows);
        const Term<T> tm = combo_term<T>(cmb, o);
        wa = valid ? tm.w0 : T(0);
        wb = valid ? tm.w1 : T(0);
        off0 = (((long)b * nsrc + tm.s0) * M + u0) * (long)ldc + y;
        off1 = (((long)b * nsrc + tm.s1) * M + u0) * (long)ldc + y;
    }
    const long ustep = (long)NT * ldc;
    // items gathered per pass over the splits: bounds the registers the
    // gather holds (FP64 with eight items took 128 registers and spilled
    // 12-20 bytes a lane, whose scratch stores added up to a fifth to the
    // written bytes; with four it takes 80: batched 512^2 x 128 adjoint
    // inverse rows 5.8 -> 5.35 ms, 100-level inverse rows 4.03 -> 3.85 ms)
    constexpr int GMAX = sizeof(T) == 8 ? 4 : 8;
    constexpr int GH = PPT > GMAX ? GMAX : PPT;
#pragma unroll
    for (int h = 0; h < PPT; h += GH) {
        cx<T> acc[GH];
#pragma unroll
        for (int i = 0; i < GH; ++i) acc[i] = cx<T>{T(0), T(0)};
        for (int sp = 0; sp < nsplit; ++sp) {
            const cx<T> *D0 = D + sp * split_stride + off0 + h * ustep;
            cx<T> x0[GH];
#pragma unroll
            for (int i = 0; i < GH; ++i) x0[i] = D0[i * ustep];
            if (two) {
                const cx<T> *D1 = D + sp * split_stride + off1 + h * ustep;
                cx<T> x1[GH];
#pragma unroll
                for (int i = 0; i < GH; ++i) x1[i] = D1[i * ustep];
#pragma unroll
                for (int i = 0; i < GH; ++i) acc[i] = add(acc[i], scale(x1[i], wb));
            }
#pragma unroll
            for (int i = 0; i < GH; ++i) acc[i] = add(acc[i], scale(x0[i], wa));
        }
#pragma unroll
        for (int i = 0; i < GH; ++i) {
            const unsigned r = r0, u = u0 + (h + i) * NT;
            T *qre = lds + (size_t)r * C::RWS;
            T *qim = qre + W;
            if (u == 0) {  // packed: X[0] = re, X[M] = im, both real
                qre[0] = acc[i].re;
                qim[0] = T(0);
                qre[F::pad(M)] = acc[i].im;
                qim[F::pad(M)] = T(0);
            } else {
                const unsigned idx = F::pad(u);
                qre[idx] = acc[i].re;
                qim[idx] = acc[i].im;
            }
        }
    }
    // the Nyquist bin of packed unit 0 (item 0 of the threads with u0 = 0)
    // from its layer chunks, when the column pass ran it apart
    if (nchunk > 0 && u0 == 0) {
        const long cstride = (long)nbatch * nsrc * ldc;
        // this row's sources in a chunk (recomputed here rather than kept
        // live through the gather)
        const long grr = gr0 + r0;
        const long gc = grr < nrows_total ? grr : 0;
        const long per_b = (long)nsub * rows;
        const int b = (int)(gc / per_b);
        const int o = (int)((gc / rows) % nsub);
        const int y = (int)(gc % rows);
        const Term<T> tm = combo_term<T>(cmb, o);
        const long noff0 = ((long)b * nsrc + tm.s0) * (long)ldc + y;
        const long noff1 = ((long)b * nsrc + tm.s1) * (long)ldc + y;
        T im = T(0);
        for (int k = 0; k < nchunk; ++k) {
            im += wa * Dny[k * cstride + noff0];
            if (two) im += wb * Dny[k * cstride + noff1];
        }
        lds[(size_t)r0 * C::RWS + F::pad(M)] = im;
    }
    const cx<T> *ftw = tw;
    if constexpr (C::TWS) {
        F::load_stage_table(lds + (size_t)TR * C::RWS, tw, twlog, threadIdx.x, C::THREADS);
        ftw = reinterpret_cast<const cx<T> *>(lds + (size_t)TR * C::RWS);
    }
    __syncthreads();

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    const long gr = gr0 + g;
    T *sre = lds + (size_t)g * C::RWS;
    T *sim = sre + W;
    const int logpx = ilog2<2 * M>::value;

    // Z[k] = Xe[k] + i Xo[k], Xe = (X[k] + conj X[M-k]) / 2,
    // Xo = (X[k] - conj X[M-k]) / (2 w^k)
    cx<T> v[PPT];
#pragma unroll
    for (int sl = 0; sl < PPT; ++sl) {
        const unsigned k = t + NT * F::elem_in(sl);
        const unsigned i1 = F::pad(k), i2 = F::pad(M - k);
        const cx<T> xk{sre[i1], sim[i1]};
        const cx<T> xm{sre[i2], -sim[i2]};
        const cx<T> xe = scale(add(xk, xm), T(0.5));
        const cx<T> xo = mul(scale(sub(xk, xm), T(0.5)), twiddle<T, true>(tw, twlog, k, logpx));
        v[sl] = cx<T>{xe.re - xo.im, xe.im + xo.re};
    }

    F::template run<true>(v, sre, sim, t, ftw, twlog);

    if (gr < nrows_total) {
        // row (b, o, y) of the output; items of a batch are out_bstride apart
        const long per_b = (long)nsub * rows;
        const long bq = gr / per_b;
        T *dst = out + bq * out_bstride + (gr - bq * per_b) * (long)nx_out;
        // (x[2j], x[2j+1]) as one vector store where the row allows it: the
        // lanes' stores then cover whole lines instead of alternate words
        const bool pairs = (nx_out & 1) == 0 && (reinterpret_cast<size_t>(dst) & (2 * sizeof(T) - 1)) == 0;
        if (pairs) {
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_out(sl);
                if (2 * j < (unsigned)nx_out) {
                    cx<T> *p = reinterpret_cast<cx<T> *>(dst + 2 * j);
                    cx<T> o{v[sl].re * sc, v[sl].im * sc};
                    if (accumulate) {
                        const cx<T> q = *p;
                        o = cx<T>{q.re + o.re, q.im + o.im};
                    }
                    *p = o;
                }
            }
        } else if (accumulate) {
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_out(sl);
                if (2 * j < (unsigned)nx_out) dst[2 * j] += v[sl].re * sc;
                if (2 * j + 1 < (unsigned)nx_out) dst[2 * j + 1] += v[sl].im * sc;
            }
        } else {
#pragma unroll
            for (int sl = 0; sl < PPT; ++sl) {
                const unsigned j = t + NT * F::elem_out(sl);
                if (2 * j < (unsigned)nx_out) dst[2 * j] = v[sl].re * sc;
                if (2 * j + 1 < (unsigned)nx_out) dst[2 * j + 1] = v[sl].im * sc;
            }
        }
    }
}

template <typename T, int M>
static int run_r2c(const void *in, long row_len, int lin, int rows, int ldc, int nsub, int src_per_b,
                   int nbatch, const RowCombo &cmb, void *out, long out_bslabs, const void *tw, int twlog,
                   hipStream_t st)
{
    using C = RowCfgF<T, M>;
    const long nrows = (long)nbatch * nsub * rows;
    if (nrows == 0) return 0;
    const long nblk = (nrows + C::TR - 1) / C::TR;
    const size_t lds = (size_t)C::TR * C::ROW_BYTES + (size_t)C::TWW * sizeof(T);
    if (lds > lds_limit()) return -3;
    if (lin <= M)
        hipLaunchKernelGGL((row_r2c_kernel<T, M, true>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                           (const T *)in, row_len, lin, rows, ldc, nsub, src_per_b, nrows, cmb, (cx<T> *)out,
                           out_bslabs > 0 ? out_bslabs : (long)nsub, (const cx<T> *)tw, twlog);
    else
        hipLaunchKernelGGL((row_r2c_kernel<T, M, false>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                           (const T *)in, row_len, lin, rows, ldc, nsub, src_per_b, nrows, cmb, (cx<T> *)out,
                           out_bslabs > 0 ? out_bslabs : (long)nsub, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int M>
static int run_c2r(const void *D, long split_stride, int nsplit, int nsrc, int rows, int ldc, int nsub,
                   int nbatch, const RowCombo &cmb, const NyqSplit &nq, void *out, long out_bstride, bool accumulate,
                   int nx_out, double scale_, const void *tw, int twlog, hipStream_t st)
{
    using C = RowCfg<T, M>;
    const long nrows = (long)nbatch * nsub * rows;
    if (nrows == 0) return 0;
    const long nblk = (nrows + C::TR - 1) / C::TR;
    const size_t lds = (size_t)C::TR * C::ROW_BYTES + (size_t)C::TWW * sizeof(T);
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((row_c2r_kernel<T, M>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                       (const cx<T> *)D, split_stride, nsplit, nsrc, rows, ldc, nsub, nrows, cmb,
                       (const T *)nq.Dny, nq.Dny ? nq.Sny : 0, nbatch, (T *)out,
                       out_bstride > 0 ? out_bstride : (long)nsub * rows * nx_out, accumulate ? 1 : 0, nx_out,
                       (T)scale_, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define GF_ROW_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048)

int launch_row_r2c(bool fp64, int px, const void *in, long row_len, int lin, int rows, int ldc,
                   int nsub, int src_per_b, int nbatch, const RowCombo &cmb, void *out, const void *tw,
                   int twlog, hipStream_t st, long out_bslabs)
{
    const int M = px / 2;
#define CASE(MM)                                                                              \
    case MM:                                                                                  \
        return fp64 ? run_r2c<double, MM>(in, row_len, lin, rows, ldc, nsub, src_per_b, nbatch, cmb, \
                                          out, out_bslabs, tw, twlog, st)                     \
                    : run_r2c<float, MM>(in, row_len, lin, rows, ldc, nsub, src_per_b, nbatch, cmb,  \
                                         out, out_bslabs, tw, twlog, st);
    switch (M) {
        GF_ROW_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_row_c2r(bool fp64, int px, const void *D, long split_stride, int nsplit, int nsrc,
                   int rows, int ldc, int nsub, int nbatch, const RowCombo &cmb, const NyqSplit &nq,
                   void *out, int nx_out, double scale_, const void *tw, int twlog, hipStream_t st,
                   long out_bstride, bool accumulate)
{
    const int M = px / 2;
#define CASE(MM)                                                                              \
    case MM:                                                                                  \
        return fp64 ? run_c2r<double, MM>(D, split_stride, nsplit, nsrc, rows, ldc, nsub, nbatch, cmb, \
                                          nq, out, out_bstride, accumulate, nx_out, scale_, tw, twlog, st) \
                    : run_c2r<float, MM>(D, split_stride, nsplit, nsrc, rows, ldc, nsub, nbatch, cmb,  \
                                         nq, out, out_bstride, accumulate, nx_out, scale_, tw, twlog, st);
    switch (M) {
        GF_ROW_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

}  // namespace gf
