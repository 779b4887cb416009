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

// Forward rows: 16 points a lane for long rows, real and imaginary parts
// exchanged one after the other through one LDS array per row; rows per
// workgroup chosen so that the transposed stores are 128-byte segments
// (16 FP32 or 8 FP64 rows) within 80 KB of LDS and 1024 threads.
template <typename T, int M>
struct RowCfgF {
    static constexpr int PPT = (M >= 1024) ? 16 : ((M >= 8) ? 8 : M);
    static constexpr int NT = M / PPT;
    static constexpr int RADIX = PPT >= 8 ? 8 : PPT;
    using FFT = BlockFFT<T, M, NT, RADIX, true, false>;
    static constexpr int W = FFT::lds_words();
    // row stride = 4 mod 64 words: the transposed reads (16 rows x 4 units per
    // wave) then fall in distinct banks
    static constexpr int WS = W + ((68 - W % 64) % 64);
    static constexpr int ROW_BYTES = WS * (int)sizeof(T);
    static constexpr int tr_calc()
    {
        int tr = 64;
        while (tr > 1 && (tr * ROW_BYTES > 80 * 1024 || tr * NT > 1024)) tr /= 2;
        return tr;
    }
    static constexpr int TR = tr_calc();
    static constexpr int THREADS = TR * NT;
};

// Inverse rows: 8 points a lane, full complex exchange.
template <typename T, int M>
struct RowCfg {
    static constexpr int PPT = (M >= 8) ? 8 : M;
    static constexpr int NT = M / PPT;
    static constexpr int RADIX = PPT;
    using FFT = BlockFFT<T, M, NT, RADIX>;
    static constexpr int W = FFT::lds_words();
    static constexpr int ROW_BYTES = 2 * W * (int)sizeof(T);
    // rows per workgroup: a power of two within 80 KB of LDS (two workgroups
    // per CU) and 1024 threads
    static constexpr int tr_calc()
    {
        int tr = 64;
        while (tr > 1 && (tr * ROW_BYTES > 80 * 1024 || tr * NT > 1024)) tr /= 2;
        return tr;
    }
    static constexpr int TR = tr_calc();
    static constexpr int THREADS = TR * NT;
};

template <typename T, int M>
__global__ void __launch_bounds__((RowCfgF<T, M>::THREADS))
    row_r2c_kernel(const T *__restrict__ in, long row_len, int lin, int rows, int ldc, int nsub, int src_per_b,
                   long nrows_total, RowCombo cmb, cx<T> *__restrict__ out,
                   const cx<T> *__restrict__ tw, int twlog)
{
    using C = RowCfgF<T, M>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, TR = C::TR, W = C::WS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    const long gr0 = (long)blockIdx.x * TR;
    const long gr = gr0 + g;
    T *sre = lds + (size_t)g * W;

    cx<T> v[PPT];
    if (gr < nrows_total) {
        const long per_b = (long)nsub * rows;
        const int b = (int)(gr / per_b);
        const int s = (int)((gr / rows) % nsub);
        const int y = (int)(gr % rows);
        int nterm = 1;
        int src0 = s, src1 = 0;
        T w0 = T(1), w1 = T(0);
        if (!cmb.identity) {
            nterm = cmb.nterm[s];
            src0 = cmb.src[s][0];
            src1 = cmb.src[s][1];
            w0 = (T)cmb.w[s][0];
            w1 = (T)cmb.w[s][1];
        }
        const T *r0 = in + (((long)b * src_per_b + src0) * rows + y) * row_len;
        const T *r1 = in + (((long)b * src_per_b + src1) * rows + y) * row_len;
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) {
            const unsigned j = t + NT * F::elem_in(sl);
            const unsigned x0 = 2 * j, x1 = 2 * j + 1;
            T re = T(0), im = T(0);
            if (nterm > 0) {
                if (x0 < (unsigned)lin) re = w0 * r0[x0];
                if (x1 < (unsigned)lin) im = w0 * r0[x1];
            }
            if (nterm > 1) {
                if (x0 < (unsigned)lin) re += w1 * r1[x0];
                if (x1 < (unsigned)lin) im += w1 * r1[x1];
            }
            v[sl] = cx<T>{re, im};
        }
    } else {
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) v[sl] = cx<T>{T(0), T(0)};
    }

    F::template run<false>(v, sre, nullptr, t, tw, twlog);

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
        const long slab = grr / rows;
        const int y = (int)(grr % rows);
        out[(slab * M + u) * (long)ldc + y] = X;
    }
}

template <typename T, int M>
__global__ void __launch_bounds__((RowCfg<T, M>::THREADS))
    row_c2r_kernel(const cx<T> *__restrict__ D, long split_stride, int nsplit, int nsrc, int rows, int ldc,
                   int nsub, long nrows_total, RowCombo cmb, T *__restrict__ out, int nx_out, T sc,
                   const cx<T> *__restrict__ tw, int twlog)
{
    using C = RowCfg<T, M>;
    using F = typename C::FFT;
    constexpr int PPT = C::PPT, NT = C::NT, TR = C::TR, W = C::W;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const long gr0 = (long)blockIdx.x * TR;
    // gather X(row)[u] transposed: consecutive lanes read consecutive rows
    for (unsigned it = threadIdx.x; it < (unsigned)(M * TR); it += C::THREADS) {
        const unsigned r = it % TR;
        const unsigned u = it / TR;
        const long grr = gr0 + r;
        cx<T> acc{T(0), T(0)};
        if (grr < nrows_total) {
            const long per_b = (long)nsub * rows;
            const int b = (int)(grr / per_b);
            const int o = (int)((grr / rows) % nsub);
            const int y = (int)(grr % rows);
            int nterm = 1;
            int srcs[2] = {o, 0};
            T ws[2] = {T(1), T(0)};
            if (!cmb.identity) {
                nterm = cmb.nterm[o];
                srcs[0] = cmb.src[o][0];
                srcs[1] = cmb.src[o][1];
                ws[0] = (T)cmb.w[o][0];
                ws[1] = (T)cmb.w[o][1];
            }
            for (int sp = 0; sp < nsplit; ++sp)
                for (int i = 0; i < nterm; ++i) {
                    const cx<T> x = D[sp * split_stride + (((long)b * nsrc + srcs[i]) * M + u) * (long)ldc + y];
                    acc = add(acc, scale(x, ws[i]));
                }
        }
        T *qre = lds + (size_t)r * 2 * W;
        T *qim = qre + W;
        if (u == 0) {  // packed: X[0] = re, X[M] = im, both real
            qre[0] = acc.re;
            qim[0] = T(0);
            qre[F::pad(M)] = acc.im;
            qim[F::pad(M)] = T(0);
        } else {
            const unsigned idx = F::pad(u);
            qre[idx] = acc.re;
            qim[idx] = acc.im;
        }
    }
    __syncthreads();

    const unsigned g = threadIdx.x / NT;
    const unsigned t = threadIdx.x % NT;
    const long gr = gr0 + g;
    T *sre = lds + (size_t)g * 2 * W;
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

    F::template run<true>(v, sre, sim, t, tw, twlog);

    if (gr < nrows_total) {
        T *dst = out + gr * (long)nx_out;
#pragma unroll
        for (int sl = 0; sl < PPT; ++sl) {
            const unsigned j = t + NT * F::elem_out(sl);
            if (2 * j < (unsigned)nx_out) dst[2 * j] = v[sl].re * sc;
            if (2 * j + 1 < (unsigned)nx_out) dst[2 * j + 1] = v[sl].im * sc;
        }
    }
}

template <typename T, int M>
static int run_r2c(const void *in, long row_len, int lin, int rows, int ldc, int nsub, int src_per_b,
                   int nbatch, const RowCombo &cmb, void *out, const void *tw, int twlog,
                   hipStream_t st)
{
    using C = RowCfgF<T, M>;
    const long nrows = (long)nbatch * nsub * rows;
    if (nrows == 0) return 0;
    const long nblk = (nrows + C::TR - 1) / C::TR;
    const size_t lds = (size_t)C::TR * C::ROW_BYTES;
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((row_r2c_kernel<T, M>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                       (const T *)in, row_len, lin, rows, ldc, nsub, src_per_b, nrows, cmb, (cx<T> *)out,
                       (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, int M>
static int run_c2r(const void *D, long split_stride, int nsplit, int nsrc, int rows, int ldc, int nsub,
                   int nbatch, const RowCombo &cmb, void *out, int nx_out, double scale_,
                   const void *tw, int twlog, hipStream_t st)
{
    using C = RowCfg<T, M>;
    const long nrows = (long)nbatch * nsub * rows;
    if (nrows == 0) return 0;
    const long nblk = (nrows + C::TR - 1) / C::TR;
    const size_t lds = (size_t)C::TR * C::ROW_BYTES;
    if (lds > lds_limit()) return -3;
    hipLaunchKernelGGL((row_c2r_kernel<T, M>), dim3((unsigned)nblk), dim3(C::THREADS), lds, st,
                       (const cx<T> *)D, split_stride, nsplit, nsrc, rows, ldc, nsub, nrows, cmb,
                       (T *)out, nx_out, (T)scale_, (const cx<T> *)tw, twlog);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define GF_ROW_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048)

int launch_row_r2c(bool fp64, int px, const void *in, long row_len, int lin, int rows, int ldc,
                   int nsub, int src_per_b, int nbatch, const RowCombo &cmb, void *out, const void *tw,
                   int twlog, hipStream_t st)
{
    const int M = px / 2;
#define CASE(MM)                                                                              \
    case MM:                                                                                  \
        return fp64 ? run_r2c<double, MM>(in, row_len, lin, rows, ldc, nsub, src_per_b, nbatch, cmb, \
                                          out, tw, twlog, st)                                 \
                    : run_r2c<float, MM>(in, row_len, lin, rows, ldc, nsub, src_per_b, nbatch, cmb,  \
                                         out, tw, twlog, st);
    switch (M) {
        GF_ROW_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

int launch_row_c2r(bool fp64, int px, const void *D, long split_stride, int nsplit, int nsrc,
                   int rows, int ldc, int nsub, int nbatch, const RowCombo &cmb, void *out, int nx_out,
                   double scale_, const void *tw, int twlog, hipStream_t st)
{
    const int M = px / 2;
#define CASE(MM)                                                                              \
    case MM:                                                                                  \
        return fp64 ? run_c2r<double, MM>(D, split_stride, nsplit, nsrc, rows, ldc, nsub, nbatch, cmb, \
                                          out, nx_out, scale_, tw, twlog, st)                 \
                    : run_c2r<float, MM>(D, split_stride, nsplit, nsrc, rows, ldc, nsub, nbatch, cmb,  \
                                         out, nx_out, scale_, tw, twlog, st);
    switch (M) {
        GF_ROW_SIZES(CASE)
    default:
        return -2;
    }
#undef CASE
}

}  // namespace gf
