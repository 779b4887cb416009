// In-register 256-point transforms of one wave (four points a lane), shared
// by the column passes and the depth transforms of the observation levels.
#pragma once

#include "gf_fft.h"

namespace gf {

// In-register transform of one wave: 256 points, four a lane, radix 4
// (gfx950 cross-lane moves instead of LDS exchanges).  The point index has
// eight bits: a lane's register slot holds two, the lane index six.  Each
// radix-4 stage works on the slot bits; between stages the slot bits trade
// places with two lane bits: v_permlane32_swap / v_permlane16_swap for lane
// bits 5 and 4, DPP for bits 3-0 (bank-masked row shifts, quad permutes).
// Forward (decimation in frequency, stages on index bits 7-6, 5-4, 3-2,
// 1-0): slot s of lane l holds n = l + 64 s on input and
// k = rev(l) + 64 s on output, rev(l) = l/16 + 4 ((l/4) mod 4) + 16 (l mod 4).
// Inverse (unnormalised): input in the forward's output layout, the lane
// bits traded in the reverse order, output m = l + 64 s.
template <typename T>
struct LaneFFT {
    static constexpr int lds_words() { return 0; }
    static constexpr int stw_entries() { return 0; }
    static constexpr int elem_in(int s) { return s; }
    static constexpr int elem_out(int s) { return s; }
    __device__ static void load_stage_table(T *, const cx<T> *, int, unsigned, unsigned) {}
};

template <typename F>
struct is_lane_fft { static constexpr bool value = false; };
template <typename T>
struct is_lane_fft<LaneFFT<T>> { static constexpr bool value = true; };

// Lane index of the forward output position: slot s of lane l holds
// frequency ws_out_lane(l) + 64 s.
template <typename F>
__device__ __forceinline__ unsigned ws_out_lane(unsigned l)
{
    if constexpr (is_lane_fft<F>::value) return (l >> 4) + 4u * ((l >> 2) & 3u) + 16u * (l & 3u);
    else return l;
}

template <int CTRL, int BANK = 0xF>
__device__ __forceinline__ unsigned dpp_word(unsigned old, unsigned x)
{
    return (unsigned)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, 0xF, BANK, false);
}

// Trade the register bit that tells a from b with lane bit B, for one
// 32-bit word: afterwards a holds the values whose lane bit B was 0 (at
// lane bit B = the old register bit), b those whose lane bit B was 1.
// `hi` is lane bit B of this lane.
template <int B>
__device__ __forceinline__ void xswap(unsigned &a, unsigned &b, bool hi)
{
    if constexpr (B == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else if constexpr (B == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else if constexpr (B == 3 || B == 2) {
        // row shifts by 2^B written only to the banks (groups of four lanes)
        // whose lane bit B is set (a: from lane l - 2^B of b) or clear (b:
        // from lane l + 2^B of a): banks 2, 3 / 0, 1 for bit 3, 1, 3 / 0, 2
        // for bit 2
        constexpr int SHR = 0x110 + (1 << B), SHL = 0x100 + (1 << B);
        constexpr int SET = B == 3 ? 0xC : 0xA, CLR = B == 3 ? 0x3 : 0x5;
        const unsigned na = dpp_word<SHR, SET>(a, b), nb = dpp_word<SHL, CLR>(b, a);
        a = na;
        b = nb;
    } else {
        // lane l ^ 1 or l ^ 2 within the quad, then a select on the lane bit
        constexpr int Q = B == 0 ? 0xB1 : 0x4E;
        const unsigned pa = dpp_word<Q>(0u, a), pb = dpp_word<Q>(0u, b);
        const unsigned na = hi ? pb : a, nb = hi ? b : pa;
        a = na;
        b = nb;
    }
}

template <int B, typename T>
__device__ __forceinline__ void cswap(cx<T> &a, cx<T> &b, bool hi)
{
    constexpr int NWD = (int)sizeof(cx<T>) / 4;
    unsigned wa[NWD], wb[NWD];
    __builtin_memcpy(wa, &a, sizeof(a));
    __builtin_memcpy(wb, &b, sizeof(b));
#pragma unroll
    for (int i = 0; i < NWD; ++i) xswap<B>(wa[i], wb[i], hi);
    __builtin_memcpy(&a, wa, sizeof(a));
    __builtin_memcpy(&b, wb, sizeof(b));
}

// slot bits 0 and 1 <-> lane bits BL and BL + 1
template <int BL, typename T>
__device__ __forceinline__ void digit_swap(cx<T> (&v)[4], unsigned lane)
{
    const bool h0 = (lane >> BL) & 1u, h1 = (lane >> (BL + 1)) & 1u;
    cswap<BL>(v[0], v[1], h0);
    cswap<BL>(v[2], v[3], h0);
    cswap<BL + 1>(v[0], v[2], h1);
    cswap<BL + 1>(v[1], v[3], h1);
}

// radix-4 butterfly over the slots: output d in slot d
template <bool INV, typename T>
__device__ __forceinline__ void radix4_slots(cx<T> (&v)[4])
{
    const cx<T> a = add(v[0], v[2]), b = sub(v[0], v[2]), c = add(v[1], v[3]), d = sub(v[1], v[3]);
    const cx<T> jd = INV ? cx<T>{-d.im, d.re} : cx<T>{d.im, -d.re};   // (+-i) d
    v[0] = add(a, c);
    v[2] = sub(a, c);
    v[1] = add(b, jd);
    v[3] = sub(b, jd);
}

// Stage twiddles of this lane, t[3 g + d - 1] for stage g and digit d = 1..3:
// forward W_256^{l d}, W_64^{(l mod 16) d}, W_16^{(l mod 4) d}; inverse the
// conjugates of W_256^{rev(l) d}, W_64^{(l/16 + 4 ((l/4) mod 4)) d},
// W_16^{(l/16) d}.  `tw` holds W_{2^twlog}^j (twlog >= 8).
template <bool INV, typename T>
__device__ __forceinline__ void lane_twiddles(cx<T> *t, const cx<T> *__restrict__ tw, int twlog, unsigned lane)
{
    const unsigned sh = (unsigned)(twlog - 8);
    const unsigned e0 = INV ? ws_out_lane<LaneFFT<T>>(lane) : lane;
    const unsigned e1 = INV ? (lane >> 4) + 4u * ((lane >> 2) & 3u) : (lane & 15u);
    const unsigned e2 = INV ? (lane >> 4) : (lane & 3u);
#pragma unroll
    for (unsigned d = 1; d < 4; ++d) {
        t[d - 1] = tw[((e0 * d) & 255u) << sh];
        t[2 + d] = tw[((4u * e1 * d) & 255u) << sh];
        t[5 + d] = tw[((16u * e2 * d) & 255u) << sh];
    }
    if (INV) {
#pragma unroll
        for (int i = 0; i < 9; ++i) t[i] = conjg(t[i]);
    }
}

template <typename T>
__device__ __forceinline__ void lane_twiddle_mul(cx<T> (&v)[4], const cx<T> *t, int g)
{
#pragma unroll
    for (int d = 1; d < 4; ++d) v[d] = mul(v[d], t[3 * g + d - 1]);
}

template <bool INV, typename T>
__device__ __forceinline__ void lane_fft(cx<T> (&v)[4], unsigned lane, const cx<T> *t)
{
    radix4_slots<INV>(v);
    lane_twiddle_mul(v, t, 0);
    if constexpr (INV) digit_swap<0>(v, lane);
    else digit_swap<4>(v, lane);
    radix4_slots<INV>(v);
    lane_twiddle_mul(v, t, 1);
    digit_swap<2>(v, lane);
    radix4_slots<INV>(v);
    lane_twiddle_mul(v, t, 2);
    if constexpr (INV) digit_swap<4>(v, lane);
    else digit_swap<0>(v, lane);
    radix4_slots<INV>(v);
}

}  // namespace gf
