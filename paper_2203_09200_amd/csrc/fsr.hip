// Block-parallel frequency selective reconstruction (FSR) for gfx950.
//
// Method: Sec. 2.1 (block-wise Fourier-domain model built from the samples of
// the block and its neighbours), Sec. 3.2 (projected samples take part in the
// model; the final overwrite uses measured samples only for D-FSR, measured
// and projected ones for R-FSR), Sec. 4 (concealed weighting 0, so every block
// is independent).  One 64-lane wavefront owns one 4x4 block and its 32x32
// support for the whole computation:
//
//   1. gather    w = a * rho^dist and w*s on the support            (registers)
//   2. DFT       Z = DFT2(w*s + i*w): 32-point passes made of one radix-2 step
//                across the two lane halves and a radix-4x4 16-point FFT in
//                registers, with a transpose through LDS between the passes
//   3. split     R = DFT(w*s), W = DFT(w) from Z(k) and Z(-k) (both inputs are
//                real); R stays in registers (16 bins per lane), W goes to a
//                32x32 LDS table
//   4. K greedy iterations: wave argmax of |R_k|^2 (first in row-major order on
//                ties) with DPP reductions, dlt = gamma R_b / W0,
//                R_k -= R_b * (gamma / W0) W(k - b) (the table is stored
//                scaled); the (b, R_b) list goes to LDS
//   5. synthesis Re sum dlt phi_b on the 16 block pixels, overwrite, store.
//
// Precision: everything from the gather to the energies is float64.  CDNA4
// issues v_fma_f64 at the rate of unpacked float32 FMA, so this costs the
// extra LDS bytes and registers only.  In float32 the transform alone gives W
// absolute errors at the scale of w*s (they share one complex FFT), and the
// argmax then departs from the float64 model in a few blocks per thousand.
//
// Register layout during 4: lane l = (h, r) with r = l & 31, h = l >> 5 holds
// the bins k = (k1, k2) = (j + 16 h, r), j = 0..15, in ascending row-major
// order along j.  W(k - b) for register j lives in table row
// ((j - b1) mod 32) xor 16h, column (r - b2) mod 32: the row part is
// wave-uniform, so each read costs one XOR of a uniform and a per-lane term.
#include "common.h"
#include "fft.h"

namespace rfsr {

namespace {

// v_max_f64 on values that are never NaN.  Written as a single instruction:
// the compiler otherwise canonicalises the bit-assembled operands first.
__device__ __forceinline__ double max_f64(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Argmax over the wave of non-negative packed energies (their bit patterns
// order like the values).  The high words are reduced first (DPP row
// reductions, one per step, and four readlanes); only when several lanes
// share the maximal high word (the first iterations, while the spectrum is
// Hermitian, and near ties) are their low words reduced as well.  Returns the
// low word of the maximum (its 5 low bits carry the row code), in `mh` its
// high word and in `owner` the first lane holding it: the lanes holding one
// packed value all own the same row, so the first is the smallest column.
__device__ __forceinline__ uint32_t wave_argmax_packed(double v, int& owner, uint32_t& mh) {
    const uint32_t hi = (uint32_t)__double2hiint(v);
    const uint32_t lo = (uint32_t)__double2loint(v);
    mh = wave_max_u32(hi);
    unsigned long long cand = __ballot(hi == mh);
    if (__popcll(cand) == 1) {
        owner = (int)__builtin_ctzll(cand);
        return (uint32_t)__builtin_amdgcn_readlane((int)lo, owner);
    }
    const uint32_t ml = wave_max_u32(hi == mh ? lo : 0u);
    cand = __ballot(hi == mh && lo == ml);
    owner = (int)__builtin_ctzll(cand);
    return ml;
}

// Energy with the bin's support row k1 packed into the 5 low mantissa bits
// as 31 - k1: the maximum over packed energies is the maximum energy with
// ties (at 2^-47 relative resolution, far below float64 rounding of the
// residual) going to the smallest k1, and k1 is read back from the maximum.
__device__ __forceinline__ double pack_energy(double e, uint32_t code) {
    const int hi = __double2hiint(e);
    const int lo = (int)(((uint32_t)__double2loint(e) & ~31u) | code);
    return __hiloint2double(hi, lo);
}

constexpr int kPlane = 33;                       // padded row length of a transpose plane

// Frame and block row of this workgroup on wavefront step `step`: a single
// frame counts rows from bi0; a batch counts the step's blocks frame after
// frame in table order.
__device__ __forceinline__ FrameJob wave_job(const Jobs<FrameJob>& js, int step, int bi0, int& bi) {
    bi = bi0 + (int)blockIdx.x;
    if (js.n == 0) return js.one;
    if (*(const_ptr<unsigned long long>)(uintptr_t)js.stamp != js.key) return js.one;   // empty job
    const_ptr<FrameJob> t = (const_ptr<FrameJob>)(uintptr_t)js.table;
    int g = (int)blockIdx.x;
    for (int f = 0; f < js.n; ++f) {
        int lo, hi;
        wave_rows(t[f].H, t[f].W, step, lo, hi);
        const int cnt = hi >= lo ? hi - lo + 1 : 0;
        if (g < cnt) {
            bi = lo + g;
            return t[f];
        }
        g -= cnt;
    }
    return js.one;   // beyond the step's blocks: empty job
}

// ------------------------------------------------------------------------
// Block DFT on the matrix cores (precision study): Z = F X F with
// F[k][m] = exp(-2 pi i k m / 32), as two 32x32x32 real GEMM stages per
// input (w*s and w) on v_mfma_f32_32x32x16_{bf16,f16}.  Every operand is
// split as x = hi + lo in the 16-bit type and a product is accumulated as
// hi*hi + hi*lo + lo*hi in float32 (lo*lo dropped).
//
// Lane layouts of the 32x32x16 MFMA (l = lane, half = l / 32):
//   A[i][k]: lane i + 32 half holds k = 8 half + t, t = 0..7
//   B[k][j]: lane j + 32 half holds k = 8 half + t
//   D[i][j]: lane j + 32 half, register r holds i = 8 (r / 4) + 4 half + r % 4
// The K index is summed over, so each stage numbers its K slots to match the
// registers the lane already holds, and stage 1 computes the frequencies in
// the order sigma(j) = 4 (j / 8) + j % 4 + 16 ((j / 4) % 2), which makes the
// stage-2 result land in the iteration layout (lane (h, c) holds
// k = (r + 16 h, c) in register r) with no data movement between stages.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int PREC> struct Mma;
template <> struct Mma<RFSR_PREC_BF16X3> {
    using V = bf16x8;
    using E = __bf16;
    static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mma<RFSR_PREC_FP16X3> {
    using V = f16x8;
    using E = _Float16;
    static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <int PREC>
struct Split {   // x = hi + lo, eight K slots
    typename Mma<PREC>::V hi, lo;
};

template <int PREC>
__device__ __forceinline__ void split_into(Split<PREC>& s, int t, float x) {
    using E = typename Mma<PREC>::E;
    const E hi = (E)x;
    s.hi[t] = hi;
    s.lo[t] = (E)(x - (float)hi);
}

// acc += a * b with split operands.
template <int PREC>
__device__ __forceinline__ f32x16 mma3(const Split<PREC>& a, const Split<PREC>& b, f32x16 acc) {
    acc = Mma<PREC>::mma(a.hi, b.hi, acc);
    acc = Mma<PREC>::mma(a.hi, b.lo, acc);
    return Mma<PREC>::mma(a.lo, b.hi, acc);
}

template <int PREC>
__device__ __forceinline__ Split<PREC> negate(const Split<PREC>& a) {
    Split<PREC> r;
    r.hi = -a.hi;
    r.lo = -a.lo;
    return r;
}

// DFT of the gathered support.  In: xs[i] = w*s, xw[i] = w at (m = i + 16 h,
// n = c).  Out (iteration layout, float64): R = DFT(w*s), W = DFT(w).
// tw: exp(-2 pi i t / 32), t = 0..31, (re, im) interleaved.
template <int PREC>
__device__ __forceinline__ void dft_mfma(const double (&xs)[16], const double (&xw)[16], int lane,
                                         const double* tw, double (&Rr)[16], double (&Ri)[16],
                                         double (&Wr)[16], double (&Wi)[16]) {
    const int j = lane & 31, half = lane >> 5;
    const int fj = 4 * (j >> 3) + (j & 3) + 16 * ((j >> 2) & 1);   // sigma(j)

    // stage 1: D1[n][j] = sum_m X[m][n] F[sigma(j)][m]; A = X^T (K slot t of
    // k-block kb is m = 16 half + 8 kb + t: the lane's own register 8 kb + t)
    f32x16 ysr = {}, ysi = {}, ywr = {}, ywi = {};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        Split<PREC> as, aw, bre, bim;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            split_into(as, t, (float)xs[8 * kb + t]);
            split_into(aw, t, (float)xw[8 * kb + t]);
            const int m = 16 * half + 8 * kb + t;
            const int e = (m * fj) & 31;
            split_into(bre, t, (float)tw[2 * e]);
            split_into(bim, t, (float)tw[2 * e + 1]);
        }
        ysr = mma3(as, bre, ysr);
        ysi = mma3(as, bim, ysi);
        ywr = mma3(aw, bre, ywr);
        ywi = mma3(aw, bim, ywi);
    }

    // stage 2: Z[sigma(i)][k2] = sum_n Y[sigma(i)][n] F[n][k2]; A = Y (the
    // lane's D1 registers 8 kb + t hold n = 16 kb + 8 (t / 4) + 4 half + t % 4)
    //   Zr = Yr C + Yi S,  Zi = Yi C - Yr S   (C = cos, S = sin of 2 pi n k2 / 32)
    f32x16 zsr = {}, zsi = {}, zwr = {}, zwi = {};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        Split<PREC> c2, s2, a_sr, a_si, a_wr, a_wi;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int n = 16 * kb + 8 * (t >> 2) + 4 * half + (t & 3);
            const int e = (n * j) & 31;
            split_into(c2, t, (float)tw[2 * e]);
            split_into(s2, t, -(float)tw[2 * e + 1]);
            split_into(a_sr, t, ysr[8 * kb + t]);
            split_into(a_si, t, ysi[8 * kb + t]);
            split_into(a_wr, t, ywr[8 * kb + t]);
            split_into(a_wi, t, ywi[8 * kb + t]);
        }
        zsr = mma3(a_sr, c2, zsr);
        zsr = mma3(a_si, s2, zsr);
        zsi = mma3(a_si, c2, zsi);
        zsi = mma3(negate(a_sr), s2, zsi);
        zwr = mma3(a_wr, c2, zwr);
        zwr = mma3(a_wi, s2, zwr);
        zwi = mma3(a_wi, c2, zwi);
        zwi = mma3(negate(a_wr), s2, zwi);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        Rr[r] = zsr[r];
        Ri[r] = zsi[r];
        Wr[r] = zwr[r];
        Wi[r] = zwi[r];
    }
}

}  // namespace

__global__ void fsr_tables_kernel(FsrTables* t, double rho, double sigma, unsigned* rerun) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kXcds && rerun) rerun[i] = 0u;   // the mixed form's lists start empty
    if (i < kSupport * kSupport) {
        const double dm = (i >> 5) - 15.5, dn = (i & 31) - 15.5;
        t->rho[i] = pow(rho, sqrt(dm * dm + dn * dn));
        // frequency distance of bin (k1, k2) from DC, both signs of k
        const int k1 = i >> 5, k2 = i & 31;
        const double f1 = min(k1, kSupport - k1), f2 = min(k2, kSupport - k2);
        t->prior[i] = sigma > 0.0 ? pow(sigma, sqrt(f1 * f1 + f2 * f2)) : 1.0;
    }
    if (i < kSupport) {
        double s, c;
        sincospi(-2.0 * i / 32.0, &s, &c);
        t->tw[2 * i] = c;
        t->tw[2 * i + 1] = s;
    }
}

// LDS (the 16 KB W table per block) caps residency at two waves per SIMD;
// telling the compiler so lets it keep the LDS reads of an iteration in flight.
// One workgroup per block of the flat block index over all the frames of
// `js`.  (A loop over several blocks per workgroup lets the compiler hoist
// per-lane tables out of it and spill; launches are cheap by comparison.)
//
// CONC (concealed weighting delta > 0, single frame): blocks run in the
// wavefront order t = 5 bi + bj, one launch per step, blockIdx.x counting
// the block rows from bi0.  A support reaches 4 blocks in each direction,
// so every raster-earlier block inside it has a smaller t (done by an
// earlier launch) and the blocks of one step never share a support.
//
// PAIRS (real-valued FSR): each iteration adds the conjugate pair dlt phi_b +
// conj(dlt) phi_-b, so the residual stays real and its spectrum Hermitian.
// The loop keeps only registers j = 0..8 of the layout (rows 0..8 and
// 16..24, which contain every row 0..16 or its conjugate), updates
// R_k -= dlt W(k - b) + conj(dlt) W(k + b) and halves dlt when b = -b.
//
// OPT (float64 FFT, independent blocks, complex bins only): bit 0 weighs the
// pick's energies with the frequency prior of `tab`, bit 1 stops a block once
// its pick's (weighted) energy falls below stop_ratio times its first.
//
// RERUN (the mixed form's float64 recomputation): the float32 pass listed
// the blocks it flagged per XCD, so the 8 lists concatenated run through the
// frame's blocks roughly in order.  Workgroup g, dispatched to XCD
// x = g mod 8, takes entry (g / 8) of the x-th eighth of that sequence: each
// XCD recomputes an equal share of neighbouring blocks (their supports
// overlap in its L2).  The grid covers every block; the workgroups beyond
// the share return at once.
template <int PREC, bool CONC, bool PAIRS, int OPT = 0, bool RERUN = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void fsr_block_kernel(
    Jobs<FrameJob> js, int total, const FsrTables* __restrict__ tab, int K, double gamma,
    double projw, int overwrite, double delta, int step, int bi0, double stop_ratio,
    unsigned* __restrict__ rerun) {
    static_assert(OPT == 0 || (PREC == RFSR_PREC_FP64 && !CONC && !PAIRS), "options: plain loop only");
    static_assert(!RERUN || (PREC == RFSR_PREC_FP64 && !CONC && !PAIRS && OPT == 0), "rerun: plain loop");
    int gb_rerun = 0;
    if constexpr (RERUN) {
        const const_ptr<unsigned> len = (const_ptr<unsigned>)(uintptr_t)rerun;
        int n = 0;
#pragma unroll
        for (int y = 0; y < kXcds; ++y) n += (int)len[y];
        const int share = (n + kXcds - 1) / kXcds;
        const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
        int e = x * share + i;   // entry of the concatenated lists
        if (i >= share || e >= n) return;
        int y = 0;
        while (e >= (int)len[y]) e -= (int)len[y++];
        gb_rerun = *(const_ptr<int>)(uintptr_t)(rerun_list(rerun, total, y) + e);
    }
    constexpr bool PRIOR = (OPT & 1) != 0, STOP = (OPT & 2) != 0;
    // W table (32 x 32 complex double); the transpose planes reuse it.  Static,
    // so its LDS base folds into the read addresses.  The (bin, dlt) list of
    // K float4 entries is dynamic LDS.
    __shared__ __align__(16) double2 s_T[32 * 32];
    __shared__ double s_tw[64];
    extern __shared__ float4 list[];
    uint8_t* smem = reinterpret_cast<uint8_t*>(s_T);

    // The frame's critical path: where other kernels share the SIMD (the next
    // frame's early motion path), the issue arbiter serves these waves first.
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x;
    const int c = lane & 31, h = lane >> 5;
    const double* __restrict__ tw = tab->tw;

    if (lane < 32) {
        s_tw[2 * lane] = tw[2 * lane];
        s_tw[2 * lane + 1] = tw[2 * lane + 1];
    }

    const int gb = RERUN ? gb_rerun : (CONC ? 0 : xcd_remap(blockIdx.x, total));
    {
        int wbi = 0;
        const FrameJob fj = CONC ? wave_job(js, step, bi0, wbi) : job_at(js, gb, &FrameJob::g_blk);
        if (fj.H == 0) return;   // empty job (stale batch table)
        const int H = fj.H, W = fj.W;
        const int64_t pitch = fj.vpitch, out_pitch = fj.pitch;
        const float* __restrict__ values = fj.values;
        const uint8_t* __restrict__ cls = fj.cls;
        float* __restrict__ out = fj.out;
        uint8_t* __restrict__ out_u8 = fj.out_u8;
        const int nbw = W >> 2;
        const int blk = gb - fj.g_blk;
        const int bi = CONC ? wbi : blk / nbw;
        const int bj = CONC ? step - 5 * bi : blk - bi * nbw;

        // 1. gather: lane (h, c) holds support rows m = i + 16 h of column c.
        //    Loads use clamped coordinates (always in bounds); positions outside
        //    the frame get weight 0.
        double zr[16], zi[16];
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
                const double rw = tab->rho[m * 32 + c];
                const double a = (k == 1u) ? 1.0 : projw;
                double wv = known ? a * rw : 0.0;
                double sv = known ? (double)v : 0.0;
                if constexpr (CONC) {
                    // an unknown pixel of a raster-earlier block: its reconstruction, weight delta
                    const bool conc = in && k == 0u && ((y >> 2) < bi || ((y >> 2) == bi && (x >> 2) < bj));
                    const float cv = out[(int64_t)yc * out_pitch + xc];   // in bounds; used only if conc
                    wv = conc ? delta * rw : wv;
                    sv = conc ? (double)cv : sv;
                }
                zr[i] = wv * sv;
                zi[i] = wv;
            }
        }

        double Rr[16], Ri[16], Wr[16], Wi[16];
        if constexpr (PREC != RFSR_PREC_FP64) {
            __syncthreads();   // s_tw
            dft_mfma<PREC>(zr, zi, lane, s_tw, Rr, Ri, Wr, Wi);
        } else {
            // 2. DFT along the support rows m (per column), transpose, DFT along n.
            double* pl = reinterpret_cast<double*>(smem);   // one 32 x 33 plane at a time
            fft32_pair(zr, zi, h, tw);                      // register k': Y[k1 = 2k'+h][n = c]
#pragma unroll
            for (int k = 0; k < 16; ++k) pl[(2 * k + h) * kPlane + c] = zr[k];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) zr[i] = pl[c * kPlane + i + 16 * h];   // row k1 = c, n = i + 16h
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; ++k) pl[(2 * k + h) * kPlane + c] = zi[k];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) zi[i] = pl[c * kPlane + i + 16 * h];
            fft32_pair(zr, zi, h, tw);                      // register j: Z[k1 = c][k2 = 2j + h]

            // 3. split Z = DFT(w s) + i DFT(w) using Z(-k), into the iteration layout
            //    k = (j + 16 h, c).
            {
                const int nc = (32 - c) & 31;
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; ++j) pl[c * kPlane + 2 * j + h] = zr[j];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k1 = j + 16 * h, nk1 = (32 - k1) & 31;
                    Wr[j] = pl[k1 * kPlane + c];      // Z.re(k)
                    Wi[j] = pl[nk1 * kPlane + nc];    // Z.re(-k)
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; ++j) pl[c * kPlane + 2 * j + h] = zi[j];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k1 = j + 16 * h, nk1 = (32 - k1) & 31;
                    const double ar = Wr[j], br = Wi[j];                                 // Z.re(k), Z.re(-k)
                    const double ai = pl[k1 * kPlane + c], bim = pl[nk1 * kPlane + nc];  // Z.im(k), Z.im(-k)
                    Rr[j] = 0.5 * (ar + br);
                    Ri[j] = 0.5 * (ai - bim);
                    Wr[j] = 0.5 * (ai + bim);
                    Wi[j] = 0.5 * (br - ar);
                }
                __syncthreads();
            }
        }
        // The table holds g W with g = gamma / W0, so that an update needs R_b
        // itself: R_k -= R_b (g W_{k-b}), and the list keeps R_b (times g at
        // synthesis).
        const double W0 = readlane_f64(Wr[0], 0);
        const double g = (W0 > 0.0) ? gamma / W0 : 0.0;
        double2* T = reinterpret_cast<double2*>(smem);
#pragma unroll
        for (int j = 0; j < 16; ++j) T[(j + 16 * h) * 32 + c] = make_double2(g * Wr[j], g * Wi[j]);
        __syncthreads();

        // 4. greedy iterations.
        constexpr int NJ = PAIRS ? 9 : 16;   // registers in the loop
        double pf[PRIOR ? 16 : 1];            // frequency prior of the lane's bins
        if constexpr (PRIOR) {
#pragma unroll
            for (int j = 0; j < 16; ++j) pf[j] = tab->prior[(j + 16 * h) * 32 + c];
        }
        double lbe = -1.0;   // packed local maximum
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            double e = fma(Rr[j], Rr[j], Ri[j] * Ri[j]);
            if constexpr (PRIOR) e *= pf[j];
            lbe = max_f64(lbe, pack_energy(e, (uint32_t)(31 - 16 * h - j)));
        }
        const uint8_t* Tb = smem;
        const uint32_t c16 = (uint32_t)c << 4, h13 = (uint32_t)h << 13;
        int kdone = K;        // iterations run (fewer after an early stop)
        double stop_at = 0.0;
        for (int it = 0; it < K; ++it) {
            int owner;
            uint32_t mhi;
            const uint32_t mlo = wave_argmax_packed(lbe, owner, mhi);
            if constexpr (STOP) {   // wave-uniform: the packed maximum itself
                const double eb = __hiloint2double((int)mhi, (int)mlo);
                if (it == 0) {
                    stop_at = stop_ratio * eb;
                } else if (eb < stop_at) {
                    kdone = it;
                    break;
                }
            }
            const int b1 = 31 - (int)(mlo & 31u);
            const int b2 = owner & 31;
            const int jb = b1 & 15;
            const double vr = Rr[jb], vi = Ri[jb];   // jb is wave-uniform: indexed register move
            double dr = readlane_f64(vr, owner);   // R_b; the table carries g
            double di = readlane_f64(vi, owner);
            if (PAIRS && (b1 & 15) == 0 && (b2 & 15) == 0) {   // b = -b: one real term
                dr *= 0.5;
                di *= 0.5;
            }
            if (lane == 0)
                list[it] = make_float4(__uint_as_float((uint32_t)(b1 * 32 + b2)), (float)dr, (float)di, 0.0f);
            const uint32_t L = ((c16 - (uint32_t)b2 * 16u) & 0x1F0u) | h13;   // per-lane column part
            lbe = -1.0;
            if constexpr (!PAIRS) {
                // issue all 16 table reads before the arithmetic so that their
                // LDS latency overlaps
                double2 wt[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t S = (uint32_t)((j - b1) & 31) << 9;   // wave-uniform row part
                    wt[j] = *reinterpret_cast<const double2*>(Tb + (S ^ L));
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const double2 wv = wt[j];
                    double xr = fma(-dr, wv.x, Rr[j]);
                    xr = fma(di, wv.y, xr);
                    double xi = fma(-dr, wv.y, Ri[j]);
                    xi = fma(-di, wv.x, xi);
                    Rr[j] = xr;
                    Ri[j] = xi;
                    double e = fma(xr, xr, xi * xi);
                    if constexpr (PRIOR) e *= pf[j];
                    lbe = max_f64(lbe, pack_energy(e, (uint32_t)(31 - 16 * h - j)));
                }
            } else {
                const uint32_t Lp = ((c16 + (uint32_t)b2 * 16u) & 0x1F0u) | h13;
                double2 wm[NJ], wp[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    wm[j] = *reinterpret_cast<const double2*>(Tb + (((uint32_t)((j - b1) & 31) << 9) ^ L));
                    wp[j] = *reinterpret_cast<const double2*>(Tb + (((uint32_t)((j + b1) & 31) << 9) ^ Lp));
                }
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    double xr = fma(-dr, wm[j].x, Rr[j]);
                    xr = fma(-dr, wp[j].x, xr);
                    xr = fma(di, wm[j].y, xr);
                    xr = fma(-di, wp[j].y, xr);
                    double xi = fma(-dr, wm[j].y, Ri[j]);
                    xi = fma(-dr, wp[j].y, xi);
                    xi = fma(-di, wm[j].x, xi);
                    xi = fma(di, wp[j].x, xi);
                    Rr[j] = xr;
                    Ri[j] = xi;
                    lbe = max_f64(lbe, pack_energy(fma(xr, xr, xi * xi), (uint32_t)(31 - 16 * h - j)));
                }
            }
        }
        __syncthreads();

        // 5. synthesis on the 16 block pixels; four lane groups split the list.
        const int p = lane & 15, q = lane >> 4;
        const int pm = 14 + (p >> 2), pn = 14 + (p & 3);
        double gr = 0.0;
        for (int it = q; it < kdone; it += 4) {
            const float4 e = list[it];
            const uint32_t bf = __float_as_uint(e.x);
            const int t = ((int)(bf >> 5) * pm + (int)(bf & 31) * pn) & 31;
            const double cs = s_tw[2 * t], sn = -s_tw[2 * t + 1];   // exp(+2 pi i t / 32)
            gr = fma((double)e.y, cs, gr);
            gr = fma(-(double)e.z, sn, gr);
        }
        gr += __shfl_xor(gr, 16);
        gr += __shfl_xor(gr, 32);
        gr *= PAIRS ? 2.0 * g : g;   // dlt = g R_b; a pair adds 2 Re(dlt phi_b)
        if (lane < 16) {
            const int y = 4 * bi + (p >> 2), x = 4 * bj + (p & 3);
            const int64_t off = (int64_t)y * pitch + x;
            const int64_t ooff = (int64_t)y * out_pitch + x;
            const uint32_t k = cls[off];
            float o = (float)gr;
            if (k == 1u || (overwrite == RFSR_RFSR && k == 2u)) o = values[off];
            out[ooff] = o;
            if (out_u8) out_u8[ooff] = (uint8_t)rintf(fminf(fmaxf(o, 0.0f), 255.0f));
        }
    }
}

hipError_t launch_fsr_tables(FsrTables* t, double rho, double prior_sigma, hipStream_t s, unsigned* rerun) {
    hipLaunchKernelGGL(fsr_tables_kernel, dim3(4), dim3(256), 0, s, t, rho, prior_sigma, rerun);
    return hipGetLastError();
}

hipError_t launch_fsr(const Jobs<FrameJob>& js, int total_blocks, const rfsr_fsr_params& p,
                      const FsrTables* tables, hipStream_t s, const FrameJob* host_frames, unsigned* rerun) {
    if (total_blocks <= 0) return hipSuccess;
    const size_t shmem = sizeof(float4) * (size_t)p.iters;
    const bool conc = p.concealed_weight > 0.0;
    if (conc && js.n != 0 && !host_frames) return hipErrorInvalidValue;
    if (conc && p.pairs) return hipErrorInvalidValue;     // not combined
    const int opt = (p.prior_sigma > 0.0 ? 1 : 0) | (p.stop_ratio > 0.0 ? 2 : 0);
    if (opt && (conc || p.pairs || p.precision != RFSR_PREC_FP64)) return hipErrorInvalidValue;
    if (p.precision == RFSR_PREC_FP32 || p.precision == RFSR_PREC_MIXED) {
        if (conc || p.pairs || opt) return hipErrorInvalidValue;
        const bool mixed = p.precision == RFSR_PREC_MIXED;
        if (mixed && !rerun) return hipErrorInvalidValue;
        MixedArgs mx;
        mx.bound = (float)p.mixed_bound;
        mx.rerun = rerun;
        mx.stats = p.rerun_blocks;
        mx.margins = p.block_margin;
        hipError_t e = launch_fsr_f32(js, total_blocks, p, tables, s, mx, mixed ? 1 : (p.block_margin ? 2 : 0));
        if (e != hipSuccess || !mixed) return e;
        // the listed blocks in float64 (after the float32 pass, in stream order)
        // every XCD gets as many workgroups as the largest share can need
        hipLaunchKernelGGL((fsr_block_kernel<RFSR_PREC_FP64, false, false, 0, true>),
                           dim3(kXcds * rerun_cap(total_blocks)), dim3(64),
                           shmem, s, js, total_blocks, tables, p.iters, p.gamma, p.proj_weight, p.overwrite, 0.0,
                           0, 0, 0.0, rerun);
        return hipGetLastError();
    }
    auto kernel = fsr_block_kernel<RFSR_PREC_FP64, false, false>;
    if (opt == 1) kernel = fsr_block_kernel<RFSR_PREC_FP64, false, false, 1>;
    else if (opt == 2) kernel = fsr_block_kernel<RFSR_PREC_FP64, false, false, 2>;
    else if (opt == 3) kernel = fsr_block_kernel<RFSR_PREC_FP64, false, false, 3>;
    else if (p.pairs) {
        kernel = fsr_block_kernel<RFSR_PREC_FP64, false, true>;
        if (p.precision == RFSR_PREC_BF16X3) kernel = fsr_block_kernel<RFSR_PREC_BF16X3, false, true>;
        else if (p.precision == RFSR_PREC_FP16X3) kernel = fsr_block_kernel<RFSR_PREC_FP16X3, false, true>;
    } else if (conc) {
        kernel = fsr_block_kernel<RFSR_PREC_FP64, true, false>;
        if (p.precision == RFSR_PREC_BF16X3) kernel = fsr_block_kernel<RFSR_PREC_BF16X3, true, false>;
        else if (p.precision == RFSR_PREC_FP16X3) kernel = fsr_block_kernel<RFSR_PREC_FP16X3, true, false>;
    } else {
        if (p.precision == RFSR_PREC_BF16X3) kernel = fsr_block_kernel<RFSR_PREC_BF16X3, false, false>;
        else if (p.precision == RFSR_PREC_FP16X3) kernel = fsr_block_kernel<RFSR_PREC_FP16X3, false, false>;
    }
    if (!conc) {
        hipLaunchKernelGGL(kernel, dim3(total_blocks), dim3(64), shmem, s, js, total_blocks, tables, p.iters,
                           p.gamma, p.proj_weight, p.overwrite, 0.0, 0, 0, p.stop_ratio, nullptr);
        return hipGetLastError();
    }
    // wavefront: step t holds the blocks with 5 bi + bj = t of every frame
    const int nf = js.n == 0 ? 1 : js.n;
    const FrameJob* fr = js.n == 0 ? &js.one : host_frames;
    int steps = 0;
    for (int f = 0; f < nf; ++f) steps = max(steps, wave_steps(fr[f].H, fr[f].W));
    for (int t = 0; t < steps; ++t) {
        int grid = 0, lo0 = 0;
        for (int f = 0; f < nf; ++f) {
            int lo, hi;
            wave_rows(fr[f].H, fr[f].W, t, lo, hi);
            if (hi >= lo) grid += hi - lo + 1;
            if (f == 0) lo0 = lo;
        }
        if (grid == 0) continue;
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), shmem, s, js, total_blocks, tables, p.iters,
                           p.gamma, p.proj_weight, p.overwrite, p.concealed_weight, t, lo0, 0.0, nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rfsr
