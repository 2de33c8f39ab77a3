// Sum of ten per-lane floats over a 64-lane wavefront (gfx950).
//
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

}  // namespace dbs
