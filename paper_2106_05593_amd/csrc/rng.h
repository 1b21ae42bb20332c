// Counter-based generator and wave reductions shared by the libmmc kernels.
#pragma once
#include "mmc_internal.h"

namespace mmc {

// ---------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (4 words), key (2 words).
// ---------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (x >> 8) * 2^-24: exact in binary32.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }

// Wave-wide sums (wave64).  Within each row of 16 lanes the partners come
// from DPP moves (VALU cross-lane operands): quad_perm [1,0,3,2] and
// [2,3,0,1] pair lanes at distance 1 and 2, row_half_mirror pairs lane i with
// 7 - i of its half-row, row_mirror lane i with 15 - i of its row; each step
// adds a lane's partial sum to its partner's, so after the four steps every
// lane of a row holds the row's sum.  The two steps across rows (16 and 32
// lanes apart) use lane permutes.  A 64-bit value moves as two 32-bit halves.
// Every lane ends with the same sum (each step adds the same two values in
// either order).
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E, kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v & 0xffffffffull), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    return __longlong_as_double((long long)dpp_u64<CTRL>((unsigned long long)__double_as_longlong(v)));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<kDppQuadXor1>(v);
    v += dpp_f64<kDppQuadXor2>(v);
    v += dpp_f64<kDppRowHalfMirror>(v);
    v += dpp_f64<kDppRowMirror>(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    v += dpp_u64<kDppQuadXor1>(v);
    v += dpp_u64<kDppQuadXor2>(v);
    v += dpp_u64<kDppRowHalfMirror>(v);
    v += dpp_u64<kDppRowMirror>(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

}  // namespace mmc
