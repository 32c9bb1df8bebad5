// Internal declarations shared by the HIP translation units of librfsr.
// gfx950 (CDNA4) only: 64-lane wavefronts, DPP row operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfsr.h"

namespace rfsr {

constexpr int kBlock = 4;      // FSR block size B
constexpr int kSupport = 32;   // FSR support / DFT size M
constexpr int kMaxIters = 1024;
constexpr int kMaxSearch = 15;
constexpr int kMaxDim = 16384;

// ---------------------------------------------------------------- wave ops --
// DPP controls (row = 16 lanes).
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xF, 0xF, false);
}

// Maximum over the 64 lanes; the result is wave-uniform.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u32<kDppQuadXor1>(v, 0u));
    v = max(v, dpp_u32<kDppQuadXor2>(v, 0u));
    v = max(v, dpp_u32<kDppRowHalfMirror>(v, 0u));
    v = max(v, dpp_u32<kDppRowMirror>(v, 0u));
    uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)max(max(a, b), max(c, d)));
}

// Minimum over the 64 lanes; the result is wave-uniform.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp_u32<kDppQuadXor1>(v, 0xFFFFFFFFu));
    v = min(v, dpp_u32<kDppQuadXor2>(v, 0xFFFFFFFFu));
    v = min(v, dpp_u32<kDppRowHalfMirror>(v, 0xFFFFFFFFu));
    v = min(v, dpp_u32<kDppRowMirror>(v, 0xFFFFFFFFu));
    uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)min(min(a, b), min(c, d)));
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Round-robin dispatch places consecutive workgroup ids on different XCDs
// (8 on MI355X, each with its own L2).  Remap so that each XCD receives a
// contiguous range of work items; neighbouring items share input data.
__device__ __forceinline__ int xcd_remap(int g, int n) {
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd;
    const int x = g % kXcd, k = g / kXcd;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// ------------------------------------------------------------ workspaces --
__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Tables used by the FSR kernel (written by fsr_tables_kernel).
struct FsrTables {
    double rho[kSupport * kSupport];  // rho ** distance to the support centre
    double tw[2 * kSupport];          // exp(-2 pi i t / 32), t = 0..31, (re, im)
};

// --------------------------------------------------------------- launches --
// Each returns hipSuccess or the launch error.
hipError_t launch_fsr_tables(FsrTables* t, double rho, hipStream_t s);
hipError_t launch_fsr(const float* values, const uint8_t* cls, int H, int W, int64_t pitch,
                      const rfsr_fsr_params& p, const FsrTables* tables, float* out,
                      uint8_t* out_u8, int64_t out_pitch, hipStream_t s);

struct MotionWs;   // defined in motion.hip
size_t motion_ws_bytes(int H, int W, const rfsr_me_params& me);
size_t frame_ws_bytes(int H, int W, int nref, const rfsr_me_params& me);

// Forward ME + check of one reference.  ws: motion workspace of
// motion_ws_bytes(); need (nullable, device H x W uint8, pitch W) restricts
// the expensive reverse test to pixels where need != 0 (decision elsewhere 0).
hipError_t run_motion_check(const uint8_t* cur, const uint8_t* cur_mask, const uint8_t* ref,
                            int H, int W, int64_t pitch, const rfsr_me_params& me,
                            int8_t* mv_a, int8_t* mv_b, int64_t mv_pitch, uint8_t* accept,
                            int64_t acc_pitch, uint16_t* cost, int64_t cost_pitch,
                            unsigned long long* counters, void* ws, bool windows_ready,
                            const uint8_t* ref_mask_for_need, hipStream_t s);

// Projection (Sec. 2.2) of up to 3 references into values/cls (pitch W).
struct ProjRef {
    const int8_t* mv_a;
    const int8_t* mv_b;
    const uint8_t* accept;
    const uint8_t* meas;
    const uint8_t* mask;
};
hipError_t launch_project(const uint8_t* cur, const uint8_t* cur_mask, int H, int W,
                          int64_t pitch, int nref, const ProjRef* refs, int64_t ipitch,
                          float* values, uint8_t* cls, hipStream_t s);

}  // namespace rfsr
