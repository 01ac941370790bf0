// Wave-level reductions shared by the gfx950 kernels (wave64, DPP moves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hough {

// One DPP step of a 64-bit maximum: v and the value the move CTRL brings
// into this lane (lanes the move does not reach keep their own).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long v) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, ROW_MASK, 0xf, false);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, ROW_MASK, 0xf, false);
    const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
    return o > v ? o : v;
}

// Largest value over the wave, returned to every lane (all 64 lanes must be
// active): row_shr 1, 2, 4, 8 leave each row's maximum in its lane 15,
// row_bcast 15 and 31 carry them up to lane 63.
__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v) {
    v = dpp_max_step<0x111, 0xf>(v);
    v = dpp_max_step<0x112, 0xf>(v);
    v = dpp_max_step<0x114, 0xf>(v);
    v = dpp_max_step<0x118, 0xf>(v);
    v = dpp_max_step<0x142, 0xa>(v);
    v = dpp_max_step<0x143, 0xc>(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

}  // namespace hough
