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

// Scalar-unit maximum of two wave-uniform values (keeps it off the vector ALU).
__device__ __forceinline__ uint32_t smax_u32(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("s_max_u32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b));
    return r;
}

// Maximum over the 64 lanes; the result is wave-uniform.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u32<kDppQuadXor1>(v, 0u));
    v = max(v, dpp_u32<kDppQuadXor2>(v, 0u));
    v = max(v, dpp_u32<kDppRowHalfMirror>(v, 0u));
    v = max(v, dpp_u32<kDppRowMirror>(v, 0u));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return smax_u32(smax_u32(a, b), smax_u32(c, d));
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

// Scratch of the mixed-precision FSR: the blocks the float32 pass flags for
// recomputation, one list per XCD (a launch of n blocks gives XCD x the
// contiguous range of xcd_remap, at most rerun_cap(n) blocks).  First 256
// bytes: the 8 list lengths; then list x at rerun_list(base, n, x).
constexpr int kXcds = 8;
__host__ __device__ inline int rerun_cap(int blocks) { return (blocks + kXcds - 1) / kXcds; }
__host__ __device__ inline size_t rerun_bytes(size_t blocks) {
    return 256 + align256(4 * (size_t)kXcds * (size_t)rerun_cap((int)blocks));
}
__device__ __forceinline__ int* rerun_list(unsigned* base, int blocks, int x) {
    return reinterpret_cast<int*>(base + 64) + (size_t)x * rerun_cap(blocks);
}

// Arguments of the float32 kernel's mixed and diagnostic modes.
struct MixedArgs {
    float bound;                  // near-tie bound a (units of 2^-24 ||R^0||_2)
    unsigned* rerun;              // rerun_bytes(total) of lists, lengths zeroed
    unsigned long long* stats;    // nullable: += the number of blocks flagged
    float* margins;               // diagnostic: per-block smallest margin
};

// Tables used by the FSR kernel (written by fsr_tables_kernel).
struct FsrTables {
    double rho[kSupport * kSupport];    // rho ** distance to the support centre
    double tw[2 * kSupport];            // exp(-2 pi i t / 32), t = 0..31, (re, im)
    double prior[kSupport * kSupport];  // frequency-weighting prior sigma ** |k| (1 when off)
};

// ------------------------------------------------------------------- jobs --
// Every kernel reads its frame or (frame, reference) pair from a job.  A
// single frame passes its jobs by value (`one`); a batch of frames passes a
// device table and each workgroup finds its job from the first-workgroup
// offsets stored in the entries (entries sorted by offset).  A batch table
// image starts with a header whose key hashes the descriptors it was built
// from; a kernel handed an image whose key differs from the launch's key
// gets an empty job (H = W = 0) and returns without touching memory.

struct TableHeader {
    unsigned long long key;
    int n_frames;
    int n_refs;
};
constexpr size_t kTableHeader = 256;

// One (frame, reference) pair of the motion path.
struct RefJob {
    const uint8_t* cur;        // measured current frame (pitch)
    const uint8_t* cur_mask;   // its mask (pitch)
    const uint8_t* ref;        // reconstruction of the reference frame (pitch)
    const uint8_t* ref_mask;   // mask of the reference, or nullptr: with it the reverse
                               // tests run only where the pixel is projectable
    int8_t* mv_a;              // outputs (opitch)
    int8_t* mv_b;
    uint8_t* accept;
    uint16_t* cost;            // best forward cost (cpitch); read by RMC/FRMC
    uint8_t* nmap_w;           // n map to write (pitch W), or nullptr
    const uint8_t* nmap;       // the frame's n map (pitch W)
    const uint2* fm;           // the frame's window plane
    int8_t* ma;                // scratch (pitch W): medians, reverse field
    int8_t* mb;
    int8_t* ra;
    int8_t* rb;
    int64_t pitch;
    int64_t opitch;
    int64_t cpitch;
    int H, W;
    int g_tile;                // first workgroup in the ME tile grid
    int g_px;                  // first workgroup in the 256-pixel grid
    int g_frmc;                // first workgroup in the FRMC-run grid
};

// One frame: window plane, projection, FSR.
struct FrameJob {
    const uint8_t* cur;
    const uint8_t* cur_mask;
    const int8_t* mv_a[3];     // per reference (opitch)
    const int8_t* mv_b[3];
    const uint8_t* accept[3];
    const uint8_t* ref_meas[3];
    const uint8_t* ref_mask[3];
    uint2* fm;                 // window plane to build, or nullptr
    float* values;             // FSR input (vpitch)
    uint8_t* cls;
    float* out;                // outputs (pitch)
    uint8_t* out_u8;           // nullable
    int64_t pitch;
    int64_t opitch;
    int64_t vpitch;
    int H, W;
    int nref;
    int g_px;                  // first workgroup in the 256-pixel grid
    int g_win;                 // first workgroup in the window-plane grid
    int g_blk;                 // first FSR block
};

template <class J>
struct Jobs {
    const J* table;                     // device table, or nullptr
    const unsigned long long* stamp;    // key stored in the table's image
    unsigned long long key;             // key expected by this launch
    int n;                              // entries in `table`; 0 selects `one`
    J one;                              // the single job; all zero with a table
};

// Tables are read through the constant address space: the job index is
// wave-uniform, so every field arrives by scalar loads and the pointers in it
// stay in SGPRs (generic pointers would turn every access that depends on the
// job into a flat access).
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;
#else   // the host pass only parses device code
template <class T>
using const_ptr = const T*;
#endif

template <class J>
__device__ __forceinline__ J job_at(const Jobs<J>& js, int g, int J::*base) {
    // a batch launch carries an all-zero `one`: the empty job for a stale image
    if (js.n == 0) return js.one;
    if (*(const_ptr<unsigned long long>)(uintptr_t)js.stamp != js.key) return js.one;
    const_ptr<J> t = (const_ptr<J>)(uintptr_t)js.table;
    int lo = 0, hi = js.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[mid].*base <= g) lo = mid; else hi = mid - 1;
    }
    return t[lo];
}

// Concealed-weighting wavefront: step t holds the blocks with 5 bi + bj = t,
// i.e. block rows [lo, hi] (empty when hi < lo); an H x W frame has
// wave_steps(H, W) steps.
__host__ __device__ inline void wave_rows(int H, int W, int t, int& lo, int& hi) {
    const int nbh = H / 4, nbw = W / 4;
    lo = t - (nbw - 1) > 0 ? (t - (nbw - 1) + 4) / 5 : 0;
    hi = nbh - 1 < t / 5 ? nbh - 1 : t / 5;
}
__host__ __device__ inline int wave_steps(int H, int W) { return 5 * (H / 4 - 1) + W / 4; }

constexpr int kPad = 16;         // border of the window planes
constexpr int kMaxFrmc = 15;     // FRMC offsets per axis in rfsr_me_params
constexpr int kMaxFrmcOffset = kPad - 2;   // a template row at a red offset stays inside the window plane

// Options of the consistency checks (from rfsr_me_params), by value to the
// kernels: raw costs, the NNC centre and an FRMC offset set of the caller's.
struct CheckOpts {
    int raw;         // compare raw S instead of S/n
    int nnc_raw;     // NNC compares the raw vector at p with the filtered neighbours
    int nf;          // FRMC offsets per axis in f[] (0: the paper's set)
    int8_t f[16];
};
constexpr int kMeTile = 16;      // forward ME tile edge
constexpr int kFrmcRun = 2048;   // pixels per FRMC workgroup (cascade)

__host__ __device__ inline int me_tiles(int H, int W) {
    return ((W + kMeTile - 1) / kMeTile) * ((H + kMeTile - 1) / kMeTile);
}
__host__ __device__ inline int px_groups(int H, int W) { return (H * W + 255) / 256; }
__host__ __device__ inline int win_groups(int H, int W) { return ((H + 2 * kPad) * (W + 2 * kPad) + 255) / 256; }
__host__ __device__ inline int frmc_groups(int H, int W) { return (H * W + kFrmcRun - 1) / kFrmcRun; }

// --------------------------------------------------------------- launches --
// Each returns hipSuccess or the launch error.
// The FSR tables; also zeroes the mixed form's list lengths at `rerun` (nullable).
hipError_t launch_fsr_tables(FsrTables* t, double rho, double prior_sigma, hipStream_t s,
                             unsigned* rerun = nullptr);
// FSR over all `total_blocks` blocks of the frames in `js`.  With a
// concealed weighting and a job table, `host_frames` is the host copy of the
// table (frame sizes for the wavefront grid).  The mixed form needs `rerun`,
// rerun_bytes(total_blocks) of scratch whose list lengths the tables launch zeroed.
hipError_t launch_fsr(const Jobs<FrameJob>& js, int total_blocks, const rfsr_fsr_params& p,
                      const FsrTables* tables, hipStream_t s, const FrameJob* host_frames = nullptr,
                      unsigned* rerun = nullptr);
// The float32 kernel (precision RFSR_PREC_FP32 and the float32 pass of
// RFSR_PREC_MIXED; independent blocks, complex bins): mode 0 plain, 1 the
// mixed form's pass, 2 plain with per-block margins (`mx`).
hipError_t launch_fsr_f32(const Jobs<FrameJob>& js, int total_blocks, const rfsr_fsr_params& p,
                          const FsrTables* tables, hipStream_t s, const MixedArgs& mx, int mode);

// Window planes of the frames in `js` (frames with fm == nullptr skipped).
hipError_t launch_windows(const Jobs<FrameJob>& js, int total_groups, hipStream_t s);
// Projection (Sec. 2.2) of the frames in `js`.
hipError_t launch_project(const Jobs<FrameJob>& js, int total_groups, hipStream_t s);
// Forward ME and the consistency check of the (frame, reference) pairs in
// `js` (window planes must exist when the check needs them).
hipError_t launch_motion(const Jobs<RefJob>& js, int total_tiles, int total_px, int total_frmc,
                         const rfsr_me_params& me, unsigned long long* counters, hipStream_t s);
bool check_needs_windows(int check);

// Quality (PSNR, mean SSIM) of a reconstruction: `partial` holds
// 2 * quality_tiles(H, W, border) doubles; `result` receives (psnr, ssim).
int quality_tiles(int H, int W, int border);
hipError_t launch_quality(const uint8_t* ref, const float* test, int H, int W, int64_t pitch, int border,
                          double* partial, double* result, hipStream_t s);

}  // namespace rfsr
