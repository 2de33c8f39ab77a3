// Cross-lane sums of ten per-lane floats (gfx950): over a whole 64-lane
// wavefront (wave_reduce10), or over each 16-lane row (row_reduce10).
//
// wave_reduce10:
// A multi-value butterfly: each exchange step halves the number of live
// registers, so ten values cost 5 + 3 swaps and 12 row-local DPP adds instead
// of 10 x 6 cross-lane shuffles.
//   1. v_permlane32_swap pairs (v0,v1) (v2,v3) (v4,v5) (v6,v7) (v8,v9):
//      afterwards register k holds partial sums of v_2k in lanes 0-31 and of
//      v_2k+1 in lanes 32-63.
//   2. v_permlane16_swap pairs those registers again; each 16-lane row of a
//      register then holds partial sums of one field:
//        s0 rows (v0, v2, v1, v3), s1 rows (v4, v6, v5, v7), s2 rows (v8, -, v9, -).
//   3. DPP row_ror 8, 4, 2, 1 sums inside every row.
// On return every lane of row r holds the totals of fields
// field0(r) = {0, 2, 1, 3}[r] in out[0], field0(r) + 4 in out[1], and for even
// rows 8 + r/2 in out[2].  Must be called with all 64 lanes active.
#pragma once

#include <hip/hip_runtime.h>

namespace dbs {

__device__ __forceinline__ float row_sum16(float x)
{
    // row_ror:n has DPP control 0x120 + n
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x128, 0xf, 0xf, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x124, 0xf, 0xf, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x122, 0xf, 0xf, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x121, 0xf, 0xf, false));
    return x;
}

__device__ __forceinline__ float swap32_add(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                             false, false);
    return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                             false, false);
    return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}

__device__ __forceinline__ void wave_reduce10(const float v[10], float out[3])
{
    const float r0 = swap32_add(v[0], v[1]);
    const float r1 = swap32_add(v[2], v[3]);
    const float r2 = swap32_add(v[4], v[5]);
    const float r3 = swap32_add(v[6], v[7]);
    const float r4 = swap32_add(v[8], v[9]);
    out[0] = row_sum16(swap16_add(r0, r1));
    out[1] = row_sum16(swap16_add(r2, r3));
    out[2] = row_sum16(swap16_add(r4, 0.0f));
}

// Field held in out[0] by the lanes of 16-lane row `row` (out[1]: +4; out[2]: 8 + row/2 for even rows).
__device__ __forceinline__ int reduce10_field0(int row) { return ((row & 1) << 1) | (row >> 1); }

// row_reduce10: the same halving idea inside each 16-lane row, with DPP
// exchanges only (no cross-row traffic).  At exchange distance 8 (row_ror:8),
// 4 (row_half_mirror), 2 and 1 (quad_perm xor 2, xor 1) a pair of registers
// (a, b) becomes one: lanes of the lower half of each exchanged pair keep
// a + partner's a, lanes of the upper half b + partner's b.  Every exchange
// pairs lanes that hold the same value with disjoint sets of summed lanes, so
// after four exchanges each lane holds a full row total.  Ten values:
// 5 + 2 + 1 + 1 halvings (3 VALU each) and 2 plain adds, 29 VALU in all.
// On return lane l of a row holds the row total of value row10_field(l)
// (-1: a duplicate, not to be stored); each value has exactly one owner.
constexpr int kDppRor8 = 0x128, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float dpp_partner(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ float halve2(float a, float b, bool upper)
{
    const float send = upper ? a : b;
    const float keep = upper ? b : a;
    return keep + dpp_partner<CTRL>(send);
}

template <int CTRL>
__device__ __forceinline__ float fold1(float a) { return a + dpp_partner<CTRL>(a); }

__device__ __forceinline__ float row_reduce10(const float v[10], int lane)
{
    const bool u8 = lane & 8, u4 = lane & 4, u2 = lane & 2, u1 = lane & 1;
    const float a0 = halve2<kDppRor8>(v[0], v[1], u8);
    const float a1 = halve2<kDppRor8>(v[2], v[3], u8);
    const float a2 = halve2<kDppRor8>(v[4], v[5], u8);
    const float a3 = halve2<kDppRor8>(v[6], v[7], u8);
    const float a4 = halve2<kDppRor8>(v[8], v[9], u8);
    const float b0 = halve2<kDppHalfMirror>(a0, a1, u4);
    const float b1 = halve2<kDppHalfMirror>(a2, a3, u4);
    const float b2 = fold1<kDppHalfMirror>(a4);
    const float c0 = halve2<kDppXor2>(b0, b1, u2);
    const float c1 = fold1<kDppXor2>(b2);
    return halve2<kDppXor1>(c0, c1, u1);
}

// Owner table of row_reduce10 (value held by lane l of a row, -1: duplicate).
__device__ __forceinline__ int row10_field(int lane)
{
    // lanes 0..15: 0, 8, 4, -, 2, -, 6, -, 1, 9, 5, -, 3, -, 7, -  (4 bits each, 15 = -)
    constexpr uint64_t kPacked = 0xf7f3f591f6f2f480ull;
    const int f = (int)((kPacked >> (4 * (lane & 15))) & 15u);
    return f == 15 ? -1 : f;
}

// Value of x held by lane src_lane (ds_bpermute: a crossbar read through the
// LDS unit, no VALU work and no LDS storage).
__device__ __forceinline__ float from_lane(float x, int src_lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src_lane << 2, __builtin_bit_cast(int, x)));
}

// kRowLanes.m[n]: 64-bit lane mask of the 16-lane rows whose bit is set in n
// (bit r: lanes 16r .. 16r+15).  A table in constant memory: a wave-uniform n
// turns into one scalar load instead of a chain of scalar shifts and masks.
struct RowLaneTable {
    uint64_t m[16];
};

constexpr RowLaneTable make_row_lane_table()
{
    RowLaneTable t{};
    for (int n = 0; n < 16; ++n)
        for (int r = 0; r < 4; ++r)
            if (n & (1 << r)) t.m[n] |= 0xFFFFull << (16 * r);
    return t;
}

static __constant__ RowLaneTable kRowLanes = make_row_lane_table();

// True in the lanes whose bit of the wave-uniform mask m is set.
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

}  // namespace dbs
