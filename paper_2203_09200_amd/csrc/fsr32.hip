// Block-parallel FSR with every step in float32 (RFSR_PREC_FP32): the plain
// float32 form of the method, kept beside the float64 kernel of fsr.hip to
// measure what float64 costs and what it buys.  Same method (Sec. 2.1; Sec.
// 3.2 for the projected samples and the overwrite; Sec. 4, concealed
// weighting 0) and the same per-wavefront structure: one 64-lane wavefront
// per 4x4 block, gather, 32x32 FFT of w*s + i*128*w, split into R = DFT(w*s)
// and W = DFT(w) (times 128), K greedy iterations, synthesis.
//
// What float32 changes:
//   * the W table is 8 KB (float2), so LDS admits four waves per SIMD instead
//     of two, and R takes 32 registers instead of 64;
//   * the argmax packs the support row into the 5 low mantissa bits of a
//     float32 energy (ties broken at 2^-18 relative instead of 2^-47) and
//     reduces one 32-bit word per lane;
//   * W is computed in the same complex FFT as w*s; packed as w*s + i*w it
//     would carry absolute errors at the scale of w*s (samples are 0..255),
//     so the packed input is w*s + i*128*w and the scale cancels in
//     gamma W / W(0);
//   * the residual carries float32 rounding through every update, so late
//     picks can still depart from the float64 model: this form is not held
//     to the 1e-3 output tolerance of the float64 one; its distance from the
//     float64 model is measured instead.
//
// Register layout of the iterations as in fsr.hip: lane (h, r) holds the bins
// k = (j + 16 h, r), j = 0..15; W(k - b) for register j sits in table row
// ((j - b1) mod 32) xor 16h, column (r - b2) mod 32.
//
// The mixed form (RFSR_PREC_MIXED) runs this kernel with a near-tie test and
// recomputes the blocks that fail it with the float64 kernel.  The float32
// residual differs from the float64 one by rounding that is dominated by the
// block's FFT: of the order of u = 2^-24 times ||R^0||_2, the norm of the
// block's initial weighted spectrum, in every bin, growing little over the
// updates.  A pick can therefore differ from the float64 model's only where
// the best and the next energy are that close.  So every iteration tests
// whether any bin other than the pick (and, while the spectrum is Hermitian,
// its conjugate partner, which ties exactly and gives the conjugate
// trajectory) has an energy within 4 a u ||R^0||_2 |R_b| of the pick's, i.e.
// |R_b| - |R_next| below about 2 a u ||R^0||_2; a block that does stops, puts
// its index in its XCD's list and leaves its outputs to the float64
// recomputation.
// `a` (rfsr_fsr_params.mixed_bound) is set well above the rounding actually
// seen at the flips (calibrated with the margin diagnostic below).  The
// per-lane second-largest packed energy, which the test needs, is tracked
// beside the maximum.
#include "common.h"
#include "fft.h"

namespace rfsr {

namespace {

// Energy with the row code 31 - k1 in the 5 low mantissa bits.  Bit patterns
// of non-negative floats order like their values, so the unsigned maximum of
// packed energies is the largest energy, ties going to the smallest k1.
__device__ __forceinline__ uint32_t pack_energy32(float e, uint32_t code) {
    return (__float_as_uint(e) & ~31u) | code;
}

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
// Three-operand unsigned max and median, written as single instructions: the
// fold below reuses its running maxima, which keeps the backend from fusing
// two-operand ones.
__device__ __forceinline__ uint32_t vmax3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t vmed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Fold four packed energies into a lane's largest (m) and second largest
// (m2): with m >= m2, the second largest of {m, m2, x, y} is
// max(m2, med3(m, x, y)); two such steps, five instructions.
__device__ __forceinline__ void fold4(uint32_t& m, uint32_t& m2, const uint32_t (&p)[4]) {
    const uint32_t ma = vmax3(m, p[0], p[1]);
    m2 = vmax3(m2, vmed3(m, p[0], p[1]), vmed3(ma, p[2], p[3]));
    m = vmax3(ma, p[2], p[3]);
}

__device__ __forceinline__ float wave_sum_f32(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

constexpr int kPlane32 = 33;   // padded row length of a transpose plane

// The packed FFT carries w in its imaginary part scaled by 2^7, so that both
// parts have the magnitude of w * s (samples are 0..255): float32 rounding
// then errs on W relative to W, not to w * s.  A power of two scales exactly.
constexpr float kWScale = 128.0f;

}  // namespace

// Four waves per SIMD fit the LDS (8 KB table + twiddles + the list).
// MODE 0: the plain float32 form.  MODE 1: the float32 pass of the mixed
// form (near-tie test; a failing block is listed in `mx` and stops).  MODE 2:
// the plain float32 form that also writes, per block, the smallest margin
// (E_b - E_next) / (4 u ||R^0||_2 |R_b|) over its iterations (a diagnostic:
// MODE 1 with bound a lists exactly the blocks whose margin is at most a).
template <int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void fsr_block_kernel_f32(
    Jobs<FrameJob> js, int total, const FsrTables* __restrict__ tab, int K, float gamma, float projw,
    int overwrite, MixedArgs mx) {
    __shared__ __align__(16) float2 s_T[32 * 32];
    __shared__ float s_tw[64];
    extern __shared__ float list[];   // K entries (bin, Re R_b, Im R_b)
    uint8_t* smem = reinterpret_cast<uint8_t*>(s_T);

    const int lane = threadIdx.x;
    const int c = lane & 31, h = lane >> 5;
    s_tw[lane] = (float)tab->tw[lane];

    const int gb = xcd_remap(blockIdx.x, total);
    const FrameJob fj = job_at(js, gb, &FrameJob::g_blk);
    if (fj.H == 0) return;   // empty job (stale batch table)
    const int H = fj.H, W = fj.W;
    const int64_t pitch = fj.vpitch, out_pitch = fj.pitch;
    const float* __restrict__ values = fj.values;
    const uint8_t* __restrict__ cls = fj.cls;
    const int nbw = W >> 2;
    const int blk = gb - fj.g_blk;
    const int bi = blk / nbw;
    const int bj = blk - bi * nbw;

    // 1. gather: lane (h, c) holds support rows m = i + 16 h of column c
    //    (clamped addresses; positions outside the frame get weight 0).
    float zr[16], zi[16];
    {
        const int y0 = 4 * bi - 14, x = 4 * bj - 14 + c;
        const bool xin = (unsigned)x < (unsigned)W;
        const int xc = min(max(x, 0), W - 1);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = i + 16 * h;
            const int y = y0 + m;
            const bool in = xin && (unsigned)y < (unsigned)H;
            const int yc = min(max(y, 0), H - 1);
            const int64_t off = (int64_t)yc * pitch + xc;
            const uint32_t k = cls[off];
            const float v = values[off];
            const bool known = in && (k == 1u || k == 2u);
            const float rw = (float)tab->rho[m * 32 + c];
            const float a = (k == 1u) ? 1.0f : projw;
            const float wv = known ? a * rw : 0.0f;
            zr[i] = wv * (known ? v : 0.0f);
            zi[i] = wv * kWScale;
        }
    }
    __syncthreads();   // s_tw

    // 2. DFT along the support rows m (per column), transpose, DFT along n.
    float Rr[16], Ri[16];
    float* pl = reinterpret_cast<float*>(smem);   // one 32 x 33 plane at a time
    fft32_pair(zr, zi, h, s_tw);                  // register k': Y[k1 = 2k'+h][n = c]
#pragma unroll
    for (int k = 0; k < 16; ++k) pl[(2 * k + h) * kPlane32 + c] = zr[k];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) zr[i] = pl[c * kPlane32 + i + 16 * h];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) pl[(2 * k + h) * kPlane32 + c] = zi[k];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) zi[i] = pl[c * kPlane32 + i + 16 * h];
    fft32_pair(zr, zi, h, s_tw);                  // register j: Z[k1 = c][k2 = 2j + h]

    // 3. split Z = DFT(w s) + i DFT(w) with Z(-k), into the iteration layout.
    float Wr[16], Wi[16];
    {
        const int nc = (32 - c) & 31;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) pl[c * kPlane32 + 2 * j + h] = zr[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k1 = j + 16 * h, nk1 = (32 - k1) & 31;
            Wr[j] = pl[k1 * kPlane32 + c];      // Z.re(k)
            Wi[j] = pl[nk1 * kPlane32 + nc];    // Z.re(-k)
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) pl[c * kPlane32 + 2 * j + h] = zi[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k1 = j + 16 * h, nk1 = (32 - k1) & 31;
            const float ar = Wr[j], br = Wi[j];
            const float ai = pl[k1 * kPlane32 + c], bim = pl[nk1 * kPlane32 + nc];
            Rr[j] = 0.5f * (ar + br);
            Ri[j] = 0.5f * (ai - bim);
            Wr[j] = 0.5f * (ai + bim);
            Wi[j] = 0.5f * (br - ar);
        }
        __syncthreads();
    }
    // near-tie scale 4 a u ||R^0||_2 (MODE 1; a = 1 for the MODE 2 margins)
    float eps4 = 0.0f;
    if constexpr (MODE != 0) {
        float e = 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j) e = fmaf(Rr[j], Rr[j], fmaf(Ri[j], Ri[j], e));
        eps4 = 4.0f * 0x1p-24f * sqrtf(wave_sum_f32(e)) * (MODE == 1 ? mx.bound : 1.0f);
    }
    // The table holds g W with g = gamma / W0; the list keeps R_b.
    const float W0 = __shfl(Wr[0], 0);                   // kWScale * W(0)
    const float g = (W0 > 0.0f) ? gamma / W0 : 0.0f;      // table: gamma * W / W(0), the scale cancels
    float2* T = reinterpret_cast<float2*>(smem);
#pragma unroll
    for (int j = 0; j < 16; ++j) T[(j + 16 * h) * 32 + c] = make_float2(g * Wr[j], g * Wi[j]);
    __syncthreads();

    // 4. greedy iterations.
    uint32_t lbe = 0u, lbe2 = 0u;   // packed local maximum and second largest (energies are >= 0)
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        uint32_t pk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            pk[q] = pack_energy32(fmaf(Rr[j + q], Rr[j + q], Ri[j + q] * Ri[j + q]), (uint32_t)(31 - 16 * h - j - q));
        if constexpr (MODE != 0) {
            fold4(lbe, lbe2, pk);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) lbe = umax(lbe, pk[q]);
        }
    }
    const uint8_t* Tb = smem;
    const uint32_t c8 = (uint32_t)c << 3, h12 = (uint32_t)h << 12;
    bool herm = true;             // residual spectrum still Hermitian (only self-conjugate picks so far)
    float mmin = __builtin_inff();
    for (int it = 0; it < K; ++it) {
        const uint32_t m = wave_max_u32(lbe);
        // lanes holding the maximal packed value share its row, so the first
        // of them holds the smallest column
        const int owner = (int)__builtin_ctzll(__ballot(lbe == m));
        const int b1 = 31 - (int)(m & 31u);
        const int b2 = owner & 31;
        const int jb = b1 & 15;
        if constexpr (MODE != 0) {
            // the largest energy of every bin but the pick and (while the
            // spectrum is Hermitian) its conjugate partner: the lane's second
            // largest in those two lanes, its largest elsewhere
            const float e1 = __uint_as_float(m);
            const int p1 = (32 - b1) & 31, p2 = (32 - b2) & 31;
            const int lane_p = ((p1 >> 4) << 5) | p2;
            const bool excl = lane == owner || (herm && lane == lane_p);
            const uint32_t other = excl ? lbe2 : lbe;
            const float r1 = __builtin_amdgcn_sqrtf(e1);   // ~1 ulp: a threshold needs no more
            if constexpr (MODE == 1) {
                const uint32_t thr = __float_as_uint(fmaxf(fmaf(-eps4, r1, e1), 0.0f));
                if (e1 > 0.0f && __ballot(other >= thr) != 0ull) {
                    if (lane == 0) {   // the float64 kernel recomputes this block
                        const int x = blockIdx.x % kXcds;
                        rerun_list(mx.rerun, total, x)[atomicAdd(mx.rerun + x, 1u)] = gb;
                        if (mx.stats) atomicAdd(mx.stats, 1ull);
                    }
                    return;
                }
            } else {
                const float e2 = __uint_as_float(wave_max_u32(other));
                if (e1 > 0.0f) mmin = fminf(mmin, (e1 - e2) / (eps4 * r1));
            }
            herm = herm && p1 == b1 && p2 == b2;
        }
        const float dr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Rr[jb]), owner));
        const float di = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Ri[jb]), owner));
        if (lane == 0) {
            list[3 * it] = __uint_as_float((uint32_t)(b1 * 32 + b2));
            list[3 * it + 1] = dr;
            list[3 * it + 2] = di;
        }
        const uint32_t L = ((c8 - (uint32_t)b2 * 8u) & 0xF8u) | h12;   // per-lane column part
        float2 wt[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t S = (uint32_t)((j - b1) & 31) << 8;   // wave-uniform row part
            wt[j] = *reinterpret_cast<const float2*>(Tb + (S ^ L));
        }
        lbe = 0u;
        lbe2 = 0u;
#pragma unroll
        for (int j = 0; j < 16; j += 4) {
            uint32_t pk[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float xr = fmaf(-dr, wt[j + q].x, Rr[j + q]);
                xr = fmaf(di, wt[j + q].y, xr);
                float xi = fmaf(-dr, wt[j + q].y, Ri[j + q]);
                xi = fmaf(-di, wt[j + q].x, xi);
                Rr[j + q] = xr;
                Ri[j + q] = xi;
                pk[q] = pack_energy32(fmaf(xr, xr, xi * xi), (uint32_t)(31 - 16 * h - j - q));
            }
            if constexpr (MODE != 0) {
                fold4(lbe, lbe2, pk);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) lbe = umax(lbe, pk[q]);
            }
        }
    }
    if constexpr (MODE == 2) {
        if (lane == 0) mx.margins[gb] = mmin;
    }
    __syncthreads();

    // 5. synthesis on the 16 block pixels; four lane groups split the list.
    const int p = lane & 15, q = lane >> 4;
    const int pm = 14 + (p >> 2), pn = 14 + (p & 3);
    float gr = 0.0f;
    for (int it = q; it < K; it += 4) {
        const uint32_t bf = __float_as_uint(list[3 * it]);
        const int t = ((int)(bf >> 5) * pm + (int)(bf & 31) * pn) & 31;
        gr = fmaf(list[3 * it + 1], s_tw[2 * t], gr);       // Re(R_b exp(+2 pi i t / 32))
        gr = fmaf(list[3 * it + 2], s_tw[2 * t + 1], gr);
    }
    gr += __shfl_xor(gr, 16);
    gr += __shfl_xor(gr, 32);
    gr *= g * kWScale;   // dlt = gamma R_b / W(0)
    if (lane < 16) {
        const int y = 4 * bi + (p >> 2), x = 4 * bj + (p & 3);
        const int64_t off = (int64_t)y * pitch + x;
        const int64_t ooff = (int64_t)y * out_pitch + x;
        const uint32_t k = cls[off];
        float o = gr;
        if (k == 1u || (overwrite == RFSR_RFSR && k == 2u)) o = values[off];
        fj.out[ooff] = o;
        if (fj.out_u8) fj.out_u8[ooff] = (uint8_t)rintf(fminf(fmaxf(o, 0.0f), 255.0f));
    }
}

hipError_t launch_fsr_f32(const Jobs<FrameJob>& js, int total_blocks, const rfsr_fsr_params& p,
                          const FsrTables* tables, hipStream_t s, const MixedArgs& mx, int mode) {
    if (total_blocks <= 0) return hipSuccess;
    // 12 bytes per list entry: with the 8.25 KB of static tables a workgroup
    // takes 19 of the CU's 320 LDS granules of 512 bytes at K = 100, so
    // sixteen (four waves per SIMD) leave room for a workgroup of another
    // kernel on the CU (the next frame's motion path on a side stream)
    const size_t shmem = 3 * sizeof(float) * (size_t)p.iters;
    auto kernel = fsr_block_kernel_f32<0>;
    if (mode == 1) kernel = fsr_block_kernel_f32<1>;
    else if (mode == 2) kernel = fsr_block_kernel_f32<2>;
    hipLaunchKernelGGL(kernel, dim3(total_blocks), dim3(64), shmem, s, js, total_blocks, tables, p.iters,
                       (float)p.gamma, (float)p.proj_weight, p.overwrite, mx);
    return hipGetLastError();
}

}  // namespace rfsr
