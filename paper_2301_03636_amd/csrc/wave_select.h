// Keys and wave-wide exchanges shared by the selection kernels (the
// argmin and top-N lists on predictions, the candidate cuts of multi-stage
// ranking): one wave of 64 lanes per kernel segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adv {

// The key of a variant orders (prediction, index) lexicographically as one unsigned
// 64-bit integer: the prediction's bits mapped to an order-preserving
// unsigned form (after folding -0 into +0) in the high half, the index in the
// low half. The minimum key is the lowest prediction, lowest index on ties.
__device__ __forceinline__ uint64_t pred_key(float p, uint32_t idx)
{
    uint32_t u = __float_as_uint(p == 0.0f ? 0.0f : p);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | idx;
}

// One step of a min-reduction over lanes through a DPP lane permutation
// inside each row of 16 lanes (the 64-bit key moves as two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_min_u64(uint64_t v)
{
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    const uint64_t o = ((uint64_t)ohi << 32) | olo;
    return o < v ? o : v;
}

__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Minimum over the 64 lanes of a wave, returned to every lane (all lanes must
// be active): swaps of neighbours and of lane pairs inside each quad, then
// the mirror images inside each half-row and row leave every lane of a row
// with the row's minimum; the four rows' minima are read out and compared.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    v = dpp_min_u64<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_min_u64<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_min_u64<0x141>(v);  // row_half_mirror
    v = dpp_min_u64<0x140>(v);  // row_mirror
    const uint64_t a = read_lane_u64(v, 0), b = read_lane_u64(v, 16);
    const uint64_t c = read_lane_u64(v, 32), d = read_lane_u64(v, 48);
    const uint64_t ab = a < b ? a : b, cd = c < d ? c : d;
    return ab < cd ? ab : cd;
}

// The key of lane (lane xor J). Inside a row of 16 lanes the exchange is a
// DPP move (xor 1 and 2: quad permutations; xor 4: the mirror image inside
// each 8-lane half-row, then each quad reversed; xor 8: a rotation of the row
// by 8); across rows it is a lane swap of the register with itself:
// v_permlane16_swap trades the odd rows of its first operand with the even
// rows of its second (so the second result holds, at an even row, the row
// after it, and the first, at an odd row, the row before it), and
// v_permlane32_swap trades the upper half of the first with the lower half
// of the second in the same way.
template <int J>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t x)
{
    const int v = (int)x;
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false);
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false);
    else if constexpr (J == 4) {
        const int m = __builtin_amdgcn_update_dpp(v, v, 0x141, 0xf, 0xf, false);  // row_half_mirror
        return (uint32_t)__builtin_amdgcn_update_dpp(m, m, 0x1B, 0xf, 0xf, false);  // quad [3,2,1,0]
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false);  // row_ror:8
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        static_assert(J == 32, "lane exchanges inside a wave of 64");
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    }
}

// The 64-bit key of lane (lane xor J), as two 32-bit exchanges.
template <int J>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t x)
{
    const uint32_t lo = xor_lane_u32<J>((uint32_t)x);
    const uint32_t hi = xor_lane_u32<J>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int J> __device__ __forceinline__ uint32_t xor_lane(uint32_t x) { return xor_lane_u32<J>(x); }
template <int J> __device__ __forceinline__ uint64_t xor_lane(uint64_t x) { return xor_lane_u64<J>(x); }

// One compare-exchange step of a bitonic sort over the wave: runs of K lanes
// alternate ascending and descending, partners are J lanes apart; the lower
// lane of a pair keeps the smaller key in an ascending run and the larger
// in a descending one.
template <int K, int J, class U>
__device__ __forceinline__ U bitonic_step(U v, int lane)
{
    const U o = xor_lane<J>(v);
    const bool keep_min = ((lane & J) == 0) == ((lane & K) == 0);
    v = ((o < v) == keep_min) ? o : v;
    if constexpr (J > 1) return bitonic_step<K, J / 2>(v, lane);
    else return v;
}

// The stages of runs of K, 2K, ... KMAX lanes: afterwards each run of KMAX
// lanes is sorted, ascending where lane & KMAX is zero (every run when
// KMAX is 64) and descending elsewhere.
template <int K, int KMAX, class U>
__device__ __forceinline__ U bitonic_from(U v, int lane)
{
    v = bitonic_step<K, K / 2>(v, lane);
    if constexpr (K < KMAX) return bitonic_from<2 * K, KMAX>(v, lane);
    else return v;
}

// Ascending bitonic sort of one 64-bit key per lane over the 64 lanes of a
// wave (lane r ends with the r-th smallest key): 21 compare-exchange steps,
// 18 of them DPP moves inside rows of 16 lanes. Every lane must be active.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v, int lane)
{
    return bitonic_from<2, 64>(v, lane);
}

// The prediction a key was made from (pred_key inverted; -0 comes back as +0).
__device__ __forceinline__ float key_pred(uint64_t key)
{
    const uint32_t u = (uint32_t)(key >> 32);
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// The threshold path of the top-N selections for a segment whose keys are
// all in registers (x[u] of every lane, ~0 where there is none): the N best
// keys (N <= 64) are found without a list per lane. One wave sort of the
// lanes' smallest prediction bits (the high halves of their minimum keys)
// gives the N-th smallest, t: N distinct eligible keys have prediction bits
// <= t, so the N best keys all do (with fewer than N eligible lanes t is the
// all-ones pattern, which no eligible key reaches, and every eligible key
// is a candidate). Where more than 64 keys share bits <= t (many equal
// predictions), a sort of the lanes' whole minimum keys gives the N-th
// smallest key itself as the bound. When at most 64 keys are at or below
// the bound they are gathered through `slot` (64 keys of LDS owned by the
// wave; each lane's at its rank among the wave's candidates, counted per
// load slot with a ballot), one more sort over the first 16, 32 or 64 lanes
// (as few as hold them all) puts them in order, lane r gets the r-th
// smallest candidate key in `v` (~0 past them) and the result is true;
// otherwise it is false and nothing is written. No eligible key is ~0 (its
// high half would be a NaN's) and none has the all-ones high half. Every
// lane must be active; N is the same in all of them.
template <int U>
__device__ __forceinline__ bool threshold_select(const uint64_t (&x)[U], int N, int lane,
                                                 uint64_t *slot, uint64_t &v)
{
    uint32_t mh = ~0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t h = (uint32_t)(x[u] >> 32);
        mh = h < mh ? h : mh;
    }
    const uint32_t t =
        (uint32_t)__builtin_amdgcn_readlane((int)bitonic_from<2, 64>(mh, lane), N - 1);
    uint64_t mask[U];
    uint32_t total = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        mask[u] = __ballot((uint32_t)(x[u] >> 32) <= t && x[u] != ~0ull);
        total += (uint32_t)__popcll(mask[u]);
    }
    if (total > 64) {
        uint64_t m = ~0ull;
#pragma unroll
        for (int u = 0; u < U; ++u) m = x[u] < m ? x[u] : m;
        const uint64_t t64 = read_lane_u64(wave_sort_u64(m, lane), N - 1);
        total = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mask[u] = __ballot(x[u] <= t64 && x[u] != ~0ull);
            total += (uint32_t)__popcll(mask[u]);
        }
        if (total > 64) return false;
    }
    uint32_t at = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mask[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask[u], 0u));
        if ((mask[u] >> lane) & 1ull) slot[at + below] = x[u];
        at += (uint32_t)__popcll(mask[u]);
    }
    // this wave's LDS writes are done before its reads below
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    v = (uint32_t)lane < total ? slot[lane] : ~0ull;
    // lanes past `total` hold ~0: the first 16 or 32 lanes sorted ascending
    // hold every candidate in order
    if (total <= 16) v = bitonic_from<2, 16>(v, lane);
    else if (total <= 32) v = bitonic_from<2, 32>(v, lane);
    else v = wave_sort_u64(v, lane);
    return true;
}

}  // namespace adv
