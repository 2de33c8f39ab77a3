// Cross-lane sums of ten per-lane floats over each 16-lane row of a
// wavefront (row_reduce10, gfx950), and the helpers that merge row totals
// across rows.
#pragma once

#include <hip/hip_runtime.h>

namespace dbs {

// row_reduce10: a multi-value butterfly inside each 16-lane row, with DPP
// exchanges only (no cross-row traffic): each exchange halves the number of
// live registers, so ten values do not cost ten separate row sums.  At
// exchange distance 8 (row_ror:8), 4 (row_half_mirror), 2 and 1 (quad_perm
// xor 2, xor 1) a pair of registers
// (a, b) becomes one: lanes of the lower half of each exchanged pair keep
// a + partner's a, lanes of the upper half b + partner's b.  Every exchange
// pairs lanes that hold the same value with disjoint sets of summed lanes, so
// after four exchanges each lane holds a full row total.  Ten values:
// 5 + 2 + 1 + 1 halvings and 2 folds; the halvings at distance 8 and 4 take
// two bank-masked DPP adds each, those at 2 and 1 three VALU: 22 VALU in all.
// On return lane l of a row holds the row total of value row10_field(l)
// (-1: a duplicate, not to be stored); each value has exactly one owner.
constexpr int kDppXor2 = 0x4E, kDppXor1 = 0xB1;  // quad_perm [2,3,0,1], [1,0,3,2]

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

// The first two exchanges pair whole 4-lane banks of a row (lanes 0-7 with
// 8-15, then 0-3 with 4-7 and 8-11 with 12-15), so each halving is two DPP
// adds whose bank masks write the lower and the upper half of the pair into
// the same register: no selects.  Written as one block: the only VALU-to-DPP
// dependences inside it are at least four instructions apart, and the
// leading and trailing s_nop 1 cover the producers before it and the DPP
// reads after it.
__device__ __forceinline__ float row_reduce10(const float v[10], int lane)
{
    const bool u2 = lane & 2, u1 = lane & 1;
    float a0, a1, a2, a3, a4, b0, b1, b2;
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %8, %8 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %0, %9, %9 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %1, %10, %10 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %1, %11, %11 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %2, %12, %12 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %2, %13, %13 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %3, %14, %14 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %3, %15, %15 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %4, %16, %16 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %4, %17, %17 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %5, %0, %0 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %5, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %6, %2, %2 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %6, %3, %3 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %7, %4, %4 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1"
        : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4), "=&v"(b0), "=&v"(b1), "=&v"(b2)
        : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]), "v"(v[8]),
          "v"(v[9]));
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
