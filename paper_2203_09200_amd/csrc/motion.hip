// Consistency-checked motion path for gfx950: pixel-wise template-matching
// motion estimation (Sec. 2.2), the reverse checks RME (Sec. 2.2), RMC and
// FRMC (Sec. 3.1.1), the nearest-neighbour check NNC (Sec. 3.1.2, Eq. (1)),
// and the projection of measured past pixels (Sec. 2.2).
//
// Template: offsets {-1,0,1,2}^2 around p.  Cost of vector v at p:
//   S(p,v) = sum_d [p+d in frame] b_t(p+d) |f_t(p+d) - Rhat(clamp(p+d+v))|
// Forward ME takes the minimum of the key (S << 16 | |v|_1 << 10 | raster(v)),
// a total order equal to (S, |v|_1, raster index of v) for R <= 15.
// Reverse costs are compared as S/n by exact cross-multiplication.
#include <string.h>

#include "common.h"

namespace rfsr {

namespace {

constexpr int kTile = kMeTile;     // forward ME tile: 16 x 16 pixels, 256 threads

__device__ __forceinline__ bool inside(int y, int x, int H, int W) {
    return (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ---------------------------------------------------------------------------
// Forward motion estimation.
//
// A workgroup handles a 16x16 pixel tile.  The reference window it needs
// ((16+3+2R) rows, clamped at the frame edge) is staged in LDS four times,
// shifted by 0..3 bytes, so that every thread reads its 4-byte aligned row
// segment with plain dword loads.  Each thread keeps the last four reference
// rows it needs in registers (one new row per vertical offset) and evaluates
// four horizontal offsets at once with v_mqsad_pk_u16_u8, which skips the
// template bytes that are 0: unmeasured template pixels are stored as 0.  A
// measured pixel of value 0 would be skipped too; waves that contain one add
// the missing |0 - ref| terms with a second masked SAD against 255.
template <int R>
struct MeGeom {
    static constexpr int NC = 2 * R + 1;            // candidates per axis
    static constexpr int NG = (NC + 3) / 4;         // groups of four horizontal offsets
    static constexpr int NV = (NC + 3) / 4 * 4;     // vertical steps, rounded up to 4
    static constexpr int ROWS = kTile + 2 + NV;     // tile rows incl. template reach and step padding
    static constexpr int ROWB = kTile + 4 * NG;     // bytes per row of one shifted copy
    static constexpr int COPY = ROWS * ROWB;        // bytes per shifted copy
};

// One vertical offset vyi: load the next reference row into r3, evaluate the
// 2R+1 horizontal offsets against rows (r0, r1, r2, r3), fold into best.
// key = (S << 16) | (|vx| << 10) + s is minimised first; the per-row part of
// the tie code, (|vy| << 10) + vyi*(2R+1), is added afterwards (no carry into
// S since the full code stays below 2^16).  Steps past the last offset
// (vyi >= 2R+1, from rounding the loop to multiples of 4) only load.
template <int R, bool BORDER, bool ZFIX>
__device__ __forceinline__ void me_step(const uint32_t (&r0)[MeGeom<R>::NG + 1],
                                        const uint32_t (&r1)[MeGeom<R>::NG + 1],
                                        const uint32_t (&r2)[MeGeom<R>::NG + 1],
                                        uint32_t (&r3)[MeGeom<R>::NG + 1],
                                        const uint8_t* __restrict__ rowbase, int ty, int vyi,
                                        const uint32_t (&t)[4], const uint32_t (&tz)[4],
                                        uint64_t zfix, int py, int px, int H, int W,
                                        uint32_t& best) {
    using G = MeGeom<R>;
    constexpr int ND = G::NG + 1;
    {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(rowbase + (ty + vyi + 3) * G::ROWB);
#pragma unroll
        for (int k = 0; k < ND; ++k) r3[k] = p[k];
    }
    if (vyi >= G::NC) return;
    const int vy = vyi - R;
    uint32_t m = 0xFFFFFFFFu;
#pragma unroll
    for (int g = 0; g < G::NG; ++g) {
        uint64_t acc = 0, acc2 = 0;
        const uint64_t s0 = ((uint64_t)r0[g + 1] << 32) | r0[g];
        const uint64_t s1 = ((uint64_t)r1[g + 1] << 32) | r1[g];
        const uint64_t s2 = ((uint64_t)r2[g + 1] << 32) | r2[g];
        const uint64_t s3 = ((uint64_t)r3[g + 1] << 32) | r3[g];
        acc = __builtin_amdgcn_mqsad_pk_u16_u8(s0, t[0], acc);
        acc = __builtin_amdgcn_mqsad_pk_u16_u8(s1, t[1], acc);
        acc = __builtin_amdgcn_mqsad_pk_u16_u8(s2, t[2], acc);
        acc = __builtin_amdgcn_mqsad_pk_u16_u8(s3, t[3], acc);
        if (ZFIX) {
            acc2 = __builtin_amdgcn_mqsad_pk_u16_u8(s0, tz[0], acc2);
            acc2 = __builtin_amdgcn_mqsad_pk_u16_u8(s1, tz[1], acc2);
            acc2 = __builtin_amdgcn_mqsad_pk_u16_u8(s2, tz[2], acc2);
            acc2 = __builtin_amdgcn_mqsad_pk_u16_u8(s3, tz[3], acc2);
            acc += zfix - acc2;
        }
        const uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = 4 * g + i;
            if (s >= G::NC) break;
            const int vx = s - R;
            const uint32_t cs = (uint32_t)((vx < 0 ? -vx : vx) << 10) + (uint32_t)s;
            uint32_t key;
            if (i == 0) key = (lo << 16) | cs;
            else if (i == 1) key = (lo & 0xFFFF0000u) | cs;
            else if (i == 2) key = (hi << 16) | cs;
            else key = (hi & 0xFFFF0000u) | cs;
            if (BORDER) {
                if ((unsigned)(px + vx) >= (unsigned)W) key = 0xFFFFFFFFu;
            }
            m = min(m, key);
        }
    }
    const uint32_t cvy = (uint32_t)((vy < 0 ? -vy : vy) << 10) + (uint32_t)(vyi * G::NC);
    bool ok = m != 0xFFFFFFFFu;
    if (BORDER) ok = ok && (unsigned)(py + vy) < (unsigned)H;
    if (ok) best = min(best, m + cvy);
}

template <int R, bool BORDER, bool ZFIX>
__device__ __forceinline__ uint32_t me_search(const uint8_t* __restrict__ rowbase, int ty,
                                              const uint32_t (&t)[4], const uint32_t (&tz)[4],
                                              uint32_t nz, int py, int px, int H, int W) {
    using G = MeGeom<R>;
    constexpr int ND = G::NG + 1;
    uint32_t a[ND], b[ND], c[ND], d[ND];
    {
        const uint32_t* p0 = reinterpret_cast<const uint32_t*>(rowbase + (ty + 0) * G::ROWB);
        const uint32_t* p1 = reinterpret_cast<const uint32_t*>(rowbase + (ty + 1) * G::ROWB);
        const uint32_t* p2 = reinterpret_cast<const uint32_t*>(rowbase + (ty + 2) * G::ROWB);
#pragma unroll
        for (int k = 0; k < ND; ++k) { a[k] = p0[k]; b[k] = p1[k]; c[k] = p2[k]; }
    }
    const uint64_t zfix = (uint64_t)(nz * 255u) * 0x0001000100010001ull;
    uint32_t best = 0xFFFFFFFFu;
#pragma unroll 1
    for (int v0 = 0; v0 < G::NC; v0 += 4) {
        me_step<R, BORDER, ZFIX>(a, b, c, d, rowbase, ty, v0 + 0, t, tz, zfix, py, px, H, W, best);
        me_step<R, BORDER, ZFIX>(b, c, d, a, rowbase, ty, v0 + 1, t, tz, zfix, py, px, H, W, best);
        me_step<R, BORDER, ZFIX>(c, d, a, b, rowbase, ty, v0 + 2, t, tz, zfix, py, px, H, W, best);
        me_step<R, BORDER, ZFIX>(d, a, b, c, rowbase, ty, v0 + 3, t, tz, zfix, py, px, H, W, best);
    }
    return best;
}

template <int R>
__global__ __launch_bounds__(256) void me_forward_kernel(Jobs<RefJob> js, int total,
                                                         unsigned long long* __restrict__ counters) {
    using G = MeGeom<R>;
    __shared__ __align__(16) uint8_t s_ref[4 * G::COPY];

    const int g = xcd_remap(blockIdx.x, total);
    const RefJob j = job_at(js, g, &RefJob::g_tile);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int H = j.H, W = j.W;
    const int64_t pitch = j.pitch;
    const int tiles_x = (W + kTile - 1) / kTile;
    const int tile = g - j.g_tile;
    const int y0 = (tile / tiles_x) * kTile, x0 = (tile % tiles_x) * kTile;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const uint8_t* __restrict__ ref = j.ref;

    // Stage the clamped reference window: the unshifted copy (and one more
    // dword per row, kept in s_tail) from global memory, then the copies
    // shifted by 1..3 bytes built from it in LDS.  Both loops are unrolled
    // with the element index clamped to the last one, so every thread issues
    // all its loads before the first wait (threads past the end rewrite the
    // last element with the same value).
    __shared__ uint32_t s_tail[G::ROWS];
    {
        constexpr int DW = G::ROWB / 4;        // dwords per copy row
        constexpr int T0 = G::ROWS * (DW + 1);
        const int gy0 = y0 - 1 - R, gx0 = x0 - 1 - R;
#pragma unroll
        for (int it = 0; it < (T0 + 255) / 256; ++it) {
            const int e = min(tid + 256 * it, T0 - 1);
            const int tr = e / (DW + 1), kd = e - tr * (DW + 1);
            const int64_t rowoff = (int64_t)clampi(gy0 + tr, 0, H - 1) * pitch;
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int gx = clampi(gx0 + 4 * kd + b, 0, W - 1);
                v |= (uint32_t)ref[rowoff + gx] << (8 * b);
            }
            if (kd < DW) reinterpret_cast<uint32_t*>(s_ref + tr * G::ROWB)[kd] = v;
            else s_tail[tr] = v;
        }
        __syncthreads();
        constexpr int T1 = 3 * G::ROWS * DW;
#pragma unroll
        for (int it = 0; it < (T1 + 255) / 256; ++it) {
            const int e = min(tid + 256 * it, T1 - 1);
            const int a = 1 + e / (G::ROWS * DW);
            const int rem = e - (a - 1) * (G::ROWS * DW);
            const int tr = rem / DW, kd = rem - tr * DW;
            const uint32_t* c0 = reinterpret_cast<const uint32_t*>(s_ref + tr * G::ROWB);
            const uint32_t lo = c0[kd];
            const uint32_t hi = kd + 1 < DW ? c0[kd + 1] : s_tail[tr];
            // bytes a..a+3 of (hi:lo): window bytes 4 kd + a .. 4 kd + a + 3
            reinterpret_cast<uint32_t*>(s_ref + a * G::COPY + tr * G::ROWB)[kd] =
                __builtin_amdgcn_alignbit(hi, lo, 8 * a);
        }
    }

    // Template of the current frame: measured bytes, 0 where unmeasured.
    // Mask and value are read at clamped (in-bounds) positions without
    // branches, so all 32 loads are in flight together.
    const int py = y0 + ty, px = x0 + tx;
    uint32_t t[4], tz[4];
    uint32_t n = 0, nz = 0;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
        uint32_t tv = 0, zv = 0;
        const int y = py - 1 + dy;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = px - 1 + i;
            const int64_t off = (int64_t)clampi(y, 0, H - 1) * pitch + clampi(x, 0, W - 1);
            const uint32_t mk = j.cur_mask[off];
            const uint32_t v = j.cur[off];
            const bool meas = inside(y, x, H, W) && mk != 0;
            tv |= (meas ? v : 0u) << (8 * i);
            zv |= (meas && v == 0 ? 0xFFu : 0u) << (8 * i);
            n += meas;
            nz += meas && v == 0;
        }
        t[dy] = tv;
        tz[dy] = zv;
    }
    __syncthreads();

    const bool interior = (y0 - R >= 0) && (y0 + kTile - 1 + R <= H - 1) && (x0 - R >= 0) &&
                          (x0 + kTile - 1 + R <= W - 1);
    const bool anyz = __any(nz != 0);
    const uint8_t* rowbase = s_ref + (tx & 3) * G::COPY + 4 * (tx >> 2);
    uint32_t best;
    if (interior) {
        best = anyz ? me_search<R, false, true>(rowbase, ty, t, tz, nz, py, px, H, W)
                    : me_search<R, false, false>(rowbase, ty, t, tz, nz, py, px, H, W);
    } else {
        best = anyz ? me_search<R, true, true>(rowbase, ty, t, tz, nz, py, px, H, W)
                    : me_search<R, true, false>(rowbase, ty, t, tz, nz, py, px, H, W);
    }

    const bool valid = py < H && px < W;
    if (valid) {
        const int raster = (int)(best & 0x3FFu);
        const int vyi = raster / G::NC, s = raster - vyi * G::NC;
        const int64_t o = (int64_t)py * j.opitch + px;
        j.mv_a[o] = (int8_t)(vyi - R);
        j.mv_b[o] = (int8_t)(s - R);
        j.cost[(int64_t)py * j.cpitch + px] = (uint16_t)(best >> 16);
        if (j.nmap_w) j.nmap_w[(int64_t)py * W + px] = (uint8_t)n;
    }
    if (counters) {
        unsigned long long cnt = 0;
        if (valid) {
            const int ny = min(R, py) + min(R, H - 1 - py) + 1;
            const int nx = min(R, px) + min(R, W - 1 - px) + 1;
            cnt = (unsigned long long)(ny * nx);
        }
        cnt = wave_sum_u64(cnt);
        if ((tid & 63) == 0) atomicAdd(counters + RFSR_CNT_FORWARD_COSTS, cnt);
    }
}

// ---------------------------------------------------------------------------
// Window planes for the reverse costs.  Entry (y, x) of the padded plane
// (rows -kPad..H+kPad-1, columns -kPad..W+kPad-1) holds, for the template row
// starting at column x-1: .x = the measured bytes of f_t (0 unmeasured or
// outside), .y = 0xFF per byte where a measurement exists.
__global__ void windows_kernel(Jobs<FrameJob> js) {
    const FrameJob j = job_at(js, (int)blockIdx.x, &FrameJob::g_win);
    if (j.H == 0) return;   // empty job (stale batch table)
    if (!j.fm) return;
    const int H = j.H, W = j.W;
    const int Wp = W + 2 * kPad, Hp = H + 2 * kPad;
    const int e = ((int)blockIdx.x - j.g_win) * 256 + (int)threadIdx.x;
    if (e >= Wp * Hp) return;
    const int y = e / Wp - kPad, x = e % Wp - kPad;
    uint32_t f = 0, m = 0;
    if ((unsigned)y < (unsigned)H) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xx = x - 1 + i;
            if ((unsigned)xx < (unsigned)W) {
                const int64_t off = (int64_t)y * j.pitch + xx;
                if (j.cur_mask[off]) {
                    f |= (uint32_t)j.cur[off] << (8 * i);
                    m |= 0xFFu << (8 * i);
                }
            }
        }
    }
    j.fm[e] = make_uint2(f, m);
}

// Reverse template cost: template r (4 rows of reference bytes at q) against
// the measured pixels of the current frame around s.
__device__ __forceinline__ uint32_t rev_cost(const RefJob& j, const uint32_t (&r)[4], int sy, int sx) {
    const int Wp = j.W + 2 * kPad;
    const uint2* p = j.fm + (int64_t)(sy - 1 + kPad) * Wp + (sx + kPad);
    uint32_t S = 0;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
        const uint2 v = p[dy * Wp];
        S = __builtin_amdgcn_sad_u8(v.x, r[dy] & v.y, S);
    }
    return S;
}

__device__ __forceinline__ void ref_template(const RefJob& j, int qy, int qx, uint32_t (&r)[4]) {
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
        const int64_t rowoff = (int64_t)clampi(qy - 1 + dy, 0, j.H - 1) * j.pitch;
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) v |= (uint32_t)j.ref[rowoff + clampi(qx - 1 + i, 0, j.W - 1)] << (8 * i);
        r[dy] = v;
    }
}

// Reverse motion field for RME: for every q the minimiser of
// (S_rev/n_rev, |u|_1, raster(u)) over u in [-R,R]^2 with q+u in the frame.
__global__ __launch_bounds__(256) void reverse_me_kernel(Jobs<RefJob> js, int R, int raw,
                                                         unsigned long long* __restrict__ counters) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    unsigned long long evals = 0;
    if (e < j.H * j.W) {
        const int qy = e / j.W, qx = e - qy * j.W;
        uint32_t r[4];
        ref_template(j, qy, qx, r);
        uint32_t bS = 0, bn = 1, bl1 = 0;
        int bu = 0, bv = 0;
        bool has = false;
        for (int uy = -R; uy <= R; ++uy) {
            const int sy = qy + uy;
            if ((unsigned)sy >= (unsigned)j.H) continue;
            for (int ux = -R; ux <= R; ++ux) {
                const int sx = qx + ux;
                if ((unsigned)sx >= (unsigned)j.W) continue;
                const uint32_t S = rev_cost(j, r, sy, sx);
                const uint32_t n = raw ? 1u : j.nmap[(int64_t)sy * j.W + sx];
                const uint32_t l1 = (uint32_t)(abs(uy) + abs(ux));
                const uint32_t lhs = S * bn, rhs = bS * n;
                ++evals;
                if (!has || lhs < rhs || (lhs == rhs && l1 < bl1)) {
                    has = true; bS = S; bn = n; bl1 = l1; bu = uy; bv = ux;
                }
            }
        }
        j.ra[e] = (int8_t)bu;
        j.rb[e] = (int8_t)bv;
    }
    if (counters) {
        evals = wave_sum_u64(evals);
        if ((threadIdx.x & 63) == 0) atomicAdd(counters + RFSR_CNT_CHECK_COSTS, evals);
    }
}

__global__ void rme_accept_kernel(Jobs<RefJob> js, unsigned long long* counters) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    unsigned long long acc_cnt = 0;
    if (e < j.H * j.W) {
        const int y = e / j.W, x = e - y * j.W;
        const int64_t o = (int64_t)y * j.opitch + x;
        const int a = j.mv_a[o], b = j.mv_b[o];
        const int q = (y + a) * j.W + (x + b);
        const bool ok = j.ra[q] == -a && j.rb[q] == -b;
        j.accept[o] = ok;
        acc_cnt = ok;
    }
    if (counters) {
        acc_cnt = wave_sum_u64(acc_cnt);
        if ((threadIdx.x & 63) == 0) atomicAdd(counters + RFSR_CNT_ACCEPTED, acc_cnt);
    }
}

// Is p a pixel whose decision matters (projectable: missing now, measured at
// p+v)?  Always true without a reference mask.
__device__ __forceinline__ bool projectable(const RefJob& j, int y, int x, int a, int b) {
    if (!j.ref_mask) return true;
    return j.cur_mask[(int64_t)y * j.pitch + x] == 0 && j.ref_mask[(int64_t)(y + a) * j.pitch + (x + b)] != 0;
}

// RMC at pixel p with vector (a, b), offsets [-rr, rr]^2: accept iff
// S(p,v)/n(p) < S(p+d, v-d)/n(p+d) (S(p,v) < S(p+d, v-d) with raw costs)
// for every red d with p+d in the frame.  Reds are tried in raster order and
// the test stops at the first loser.  evals counts the red costs evaluated.
__device__ __forceinline__ bool rmc_test(const RefJob& j, int py, int px, int a, int b, int rr, int raw,
                                         unsigned long long& evals) {
    uint32_t r[4];
    ref_template(j, py + a, px + b, r);
    const uint32_t Sg = j.cost[(int64_t)py * j.cpitch + px];
    const uint32_t ng = raw ? 1u : j.nmap[(int64_t)py * j.W + px];
    bool ok = true;
    for (int dy = -rr; dy <= rr && ok; ++dy) {
        const int sy = py + dy;
        if ((unsigned)sy >= (unsigned)j.H) continue;
        for (int dx = -rr; dx <= rr; ++dx) {
            const int sx = px + dx;
            if ((dy | dx) == 0 || (unsigned)sx >= (unsigned)j.W) continue;
            const uint32_t S = rev_cost(j, r, sy, sx);
            const uint32_t n = raw ? 1u : j.nmap[(int64_t)sy * j.W + sx];
            ++evals;
            if (S * ng <= Sg * n) { ok = false; break; }
        }
    }
    return ok;
}

// Red candidates of one FRMC offset row sy for a caller's offset set: true if
// one of the candidates (sy, px + dxs[ix]) whose bit is set in `active` and
// that lies in the frame is not worse than the green (reads up to +-kPad
// columns stay inside the padded window plane; an out-of-frame candidate
// only drops out of the comparison).  evals counts the in-frame reds.
template <int N>
__device__ __forceinline__ bool frmc_row_loses(const RefJob& j, const uint32_t (&r)[4], int sy, int px,
                                               const int (&dxs)[N], uint32_t active, uint32_t Sg,
                                               uint32_t ng, int raw, unsigned long long& evals) {
    const int Wp = j.W + 2 * kPad;
    const uint2* row = j.fm + (int64_t)(sy - 1 + kPad) * Wp + (px + kPad);
    const uint8_t* nrow = j.nmap + (int64_t)sy * j.W;
    bool lose = false;
#pragma unroll
    for (int ix = 0; ix < N; ++ix) {
        if (!((active >> ix) & 1u)) continue;
        const int dx = dxs[ix];
        const int sx = px + dx;
        const bool in = (unsigned)sx < (unsigned)j.W;
        uint32_t S = 0;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            const uint2 v = row[dy * Wp + dx];
            S = __builtin_amdgcn_sad_u8(v.x, r[dy] & v.y, S);
        }
        const uint32_t n = raw ? 1u : nrow[clampi(sx, 0, j.W - 1)];
        evals += in;
        lose |= in & (S * ng <= Sg * n);
    }
    return lose;
}

// FRMC at pixel p with vector (a, b): the acceptance rule of rmc_test over
// the offsets {-7,-3,-1,0,1,3,7}^2, or with CUSTOM over the caller's set
// o.f[0..o.nf-1]^2, organised for memory-level parallelism: the red
// candidates of one offset row are evaluated together (for the paper's set
// their 28 window reads have no branch between them: the padded window plane
// covers offsets up to +-kPad, and an out-of-frame candidate only drops out
// of the comparison), and the test stops after the first row that holds a
// loser; evals counts the in-frame red costs of the rows evaluated.
template <bool CUSTOM>
__device__ __forceinline__ bool frmc_test(const RefJob& j, int py, int px, int a, int b, const CheckOpts& o,
                                          unsigned long long& evals) {
    static_assert(kPad >= 7 + 2 && kMaxFrmcOffset + 2 <= kPad,
                  "window plane border must cover the FRMC offsets and the template");
    uint32_t r[4];
    ref_template(j, py + a, px + b, r);
    const uint32_t Sg = j.cost[(int64_t)py * j.cpitch + px];
    const uint32_t ng = o.raw ? 1u : j.nmap[(int64_t)py * j.W + px];
    if constexpr (!CUSTOM) {
        constexpr int kOff[7] = {-7, -3, -1, 0, 1, 3, 7};
        const int Wp = j.W + 2 * kPad;
#pragma unroll
        for (int iy = 0; iy < 7; ++iy) {
            const int sy = py + kOff[iy];
            if ((unsigned)sy >= (unsigned)j.H) continue;
            const uint2* row = j.fm + (int64_t)(sy - 1 + kPad) * Wp + (px + kPad);
            const uint8_t* nrow = j.nmap + (int64_t)sy * j.W;
            bool lose = false;
#pragma unroll
            for (int ix = 0; ix < 7; ++ix) {
                if (iy == 3 && ix == 3) continue;   // the green candidate
                const int dx = kOff[ix];
                const int sx = px + dx;
                const bool in = (unsigned)sx < (unsigned)j.W;
                uint32_t S = 0;
#pragma unroll
                for (int dy = 0; dy < 4; ++dy) {
                    const uint2 v = row[dy * Wp + dx];
                    S = __builtin_amdgcn_sad_u8(v.x, r[dy] & v.y, S);
                }
                const uint32_t n = o.raw ? 1u : nrow[clampi(sx, 0, j.W - 1)];
                evals += in;
                lose |= in & (S * ng <= Sg * n);   // no short circuit: the reads stay unconditional
            }
            if (lose) return false;
        }
    } else {
        // the caller's offsets, copied with constant indices (entries beyond
        // o.nf are inactive and read column offset 0, inside the plane)
        int off[kMaxFrmc];
        uint32_t all = 0, green = 0;
#pragma unroll
        for (int i = 0; i < kMaxFrmc; ++i) {
            off[i] = i < o.nf ? (int)o.f[i] : 0;
            all |= (i < o.nf ? 1u : 0u) << i;
            green |= (i < o.nf && o.f[i] == 0 ? 1u : 0u) << i;
        }
#pragma unroll
        for (int iy = 0; iy < kMaxFrmc; ++iy) {
            if (iy >= o.nf) break;
            const int sy = py + off[iy];
            if ((unsigned)sy >= (unsigned)j.H) continue;
            const uint32_t active = off[iy] == 0 ? all & ~green : all;
            if (frmc_row_loses(j, r, sy, px, off, active, Sg, ng, o.raw, evals)) return false;
        }
    }
    return true;
}

// RMC / FRMC over every pixel (stand-alone checks); with a reference mask
// only projectable pixels are tested and the decision elsewhere is 0.
template <bool DENSE, bool CUSTOM>
__global__ __launch_bounds__(256) void rmc_kernel(Jobs<RefJob> js, int rr, CheckOpts opts,
                                                  unsigned long long* __restrict__ counters) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    unsigned long long evals = 0, checked = 0, accepted = 0;
    if (e < j.H * j.W) {
        const int py = e / j.W, px = e - py * j.W;
        const int64_t o = (int64_t)py * j.opitch + px;
        const int a = j.mv_a[o], b = j.mv_b[o];
        bool ok = projectable(j, py, px, a, b);
        if (ok) {
            checked = 1;
            ok = DENSE ? rmc_test(j, py, px, a, b, rr, opts.raw, evals)
                       : frmc_test<CUSTOM>(j, py, px, a, b, opts, evals);
        }
        j.accept[o] = ok;
        accepted = ok;
    }
    if (counters) {
        evals = wave_sum_u64(evals);
        checked = wave_sum_u64(checked);
        accepted = wave_sum_u64(accepted);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(counters + RFSR_CNT_CHECK_COSTS, evals);
            atomicAdd(counters + RFSR_CNT_CHECKED_PIXELS, checked);
            atomicAdd(counters + RFSR_CNT_ACCEPTED, accepted);
        }
    }
}

// FRMC after NNC (the cascade).  A workgroup owns a run of kFrmcRun raster
// pixels: it collects the pixels that need the test (NNC accepted and, with a
// reference mask, projectable) into an LDS list, then runs FRMC over that
// list with all its threads, so that waves stay full although most pixels
// need no test.  Every pixel of the run gets its decision written.
template <bool CUSTOM>
__global__ __launch_bounds__(256) void frmc_tile_kernel(Jobs<RefJob> js, CheckOpts opts,
                                                        unsigned long long* __restrict__ counters) {
    __shared__ int s_list[kFrmcRun];
    __shared__ unsigned s_n;
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_frmc);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int tid = threadIdx.x;
    const int npx = j.H * j.W;
    const int e0 = ((int)blockIdx.x - j.g_frmc) * kFrmcRun;
    if (tid == 0) s_n = 0u;
    __syncthreads();
    unsigned long long checked = 0;
    for (int k = 0; k < kFrmcRun / 256; ++k) {
        const int e = e0 + k * 256 + tid;
        bool need = false;
        if (e < npx) {
            const int y = e / j.W, x = e - y * j.W;
            const int64_t o = (int64_t)y * j.opitch + x;
            need = j.accept[o] != 0;   // NNC decision
            if (need) need = projectable(j, y, x, j.mv_a[o], j.mv_b[o]);
            if (!need) j.accept[o] = 0;
        }
        // wave-aggregated append to the LDS list
        const unsigned long long m = __ballot(need);
        const int lane = tid & 63;
        unsigned base = 0;
        if (lane == 0 && m) base = atomicAdd(&s_n, (unsigned)__popcll(m));
        base = __shfl(base, 0);
        if (need) s_list[base + __popcll(m & ((1ull << lane) - 1ull))] = e;
        checked += need;
    }
    __syncthreads();
    const unsigned n = s_n;
    unsigned long long evals = 0, accepted = 0;
    for (unsigned i = tid; i < n; i += 256) {
        const int e = s_list[i];
        const int py = e / j.W, px = e - py * j.W;
        const int64_t o = (int64_t)py * j.opitch + px;
        const bool ok = frmc_test<CUSTOM>(j, py, px, j.mv_a[o], j.mv_b[o], opts, evals);
        j.accept[o] = ok;
        accepted += ok;
    }
    if (counters) {
        evals = wave_sum_u64(evals);
        accepted = wave_sum_u64(accepted);
        checked = wave_sum_u64(checked);
        if ((tid & 63) == 0) {
            atomicAdd(counters + RFSR_CNT_CHECK_COSTS, evals);
            atomicAdd(counters + RFSR_CNT_ACCEPTED, accepted);
            atomicAdd(counters + RFSR_CNT_CHECKED_PIXELS, checked);
        }
    }
}

// ----------------------------------------------------------------- NNC ----
__device__ __forceinline__ void sort2(int& a, int& b) {
    const int lo = min(a, b), hi = max(a, b);
    a = lo; b = hi;
}
__device__ __forceinline__ int med3(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// Median of a 3x3 neighbourhood: sort each row, then the median of
// (largest row minimum, median of row medians, smallest row maximum).
__device__ __forceinline__ int median9(int (&v)[9]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        sort2(v[3 * r], v[3 * r + 1]);
        sort2(v[3 * r + 1], v[3 * r + 2]);
        sort2(v[3 * r], v[3 * r + 1]);
    }
    const int lo = max(max(v[0], v[3]), v[6]);
    const int hi = min(min(v[2], v[5]), v[8]);
    const int md = med3(v[1], v[4], v[7]);
    return med3(lo, md, hi);
}

__global__ void median_kernel(Jobs<RefJob> js) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    const int H = j.H, W = j.W;
    if (e >= H * W) return;
    const int y = e / W, x = e - y * W;
    int va[9], vb[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const int64_t ro = (int64_t)clampi(y - 1 + dy, 0, H - 1) * j.opitch;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int xx = clampi(x - 1 + dx, 0, W - 1);
            va[3 * dy + dx] = j.mv_a[ro + xx];
            vb[3 * dy + dx] = j.mv_b[ro + xx];
        }
    }
    j.ma[e] = (int8_t)median9(va);
    j.mb[e] = (int8_t)median9(vb);
}

// NNC decision (the cascade's FRMC reads it back from `accept`).  With
// center_raw the raw vector at p is compared with the filtered neighbours.
__global__ void nnc_kernel(Jobs<RefJob> js, int center_raw, unsigned long long* counters, bool count) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    const int H = j.H, W = j.W;
    unsigned long long acc_cnt = 0;
    if (e < H * W) {
        const int y = e / W, x = e - y * W;
        const int8_t* __restrict__ ma = j.ma;
        const int8_t* __restrict__ mb = j.mb;
        const int64_t o = (int64_t)y * j.opitch + x;
        const int a = center_raw ? (int)j.mv_a[o] : (int)ma[e];
        const int b = center_raw ? (int)j.mv_b[o] : (int)mb[e];
        bool ok = true;
        if (y > 0) ok &= abs(a - ma[e - W]) + abs(b - mb[e - W]) <= 1;
        if (y < H - 1) ok &= abs(a - ma[e + W]) + abs(b - mb[e + W]) <= 1;
        if (x > 0) ok &= abs(a - ma[e - 1]) + abs(b - mb[e - 1]) <= 1;
        if (x < W - 1) ok &= abs(a - ma[e + 1]) + abs(b - mb[e + 1]) <= 1;
        j.accept[o] = ok;
        acc_cnt = ok;
    }
    if (count && counters) {
        acc_cnt = wave_sum_u64(acc_cnt);
        if ((threadIdx.x & 63) == 0) atomicAdd(counters + RFSR_CNT_ACCEPTED, acc_cnt);
    }
}

__global__ void accept_all_kernel(Jobs<RefJob> js, unsigned long long* counters) {
    const RefJob j = job_at(js, (int)blockIdx.x, &RefJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    unsigned long long acc_cnt = 0;
    if (e < j.H * j.W) {
        j.accept[(int64_t)(e / j.W) * j.opitch + (e % j.W)] = 1;
        acc_cnt = 1;
    }
    if (counters) {
        acc_cnt = wave_sum_u64(acc_cnt);
        if ((threadIdx.x & 63) == 0) atomicAdd(counters + RFSR_CNT_ACCEPTED, acc_cnt);
    }
}

// ----------------------------------------------------------- projection ----
__global__ void project_kernel(Jobs<FrameJob> js) {
    const FrameJob j = job_at(js, (int)blockIdx.x, &FrameJob::g_px);
    if (j.H == 0) return;   // empty job (stale batch table)
    const int e = ((int)blockIdx.x - j.g_px) * 256 + (int)threadIdx.x;
    const int W = j.W;
    if (e >= j.H * W) return;
    const int y = e / W, x = e - y * W;
    const int64_t off = (int64_t)y * j.pitch + x;
    if (j.cur_mask[off]) {
        j.values[e] = (float)j.cur[off];
        j.cls[e] = 1;
        return;
    }
    uint32_t total = 0, count = 0;
    const int64_t io = (int64_t)y * j.opitch + x;
#pragma unroll
    for (int k = 0; k < 3; ++k) {   // constant indices keep the job's arrays in registers
        if (k >= j.nref || !j.accept[k][io]) continue;
        const int qy = y + j.mv_a[k][io], qx = x + j.mv_b[k][io];
        const int64_t qo = (int64_t)qy * j.pitch + qx;
        if (j.ref_mask[k][qo]) {
            total += j.ref_meas[k][qo];
            count += 1;
        }
    }
    j.values[e] = count ? (float)total / (float)count : 0.0f;
    j.cls[e] = count ? 2 : 0;
}

// ------------------------------------------------------------- dispatch ----
template <int R>
hipError_t launch_me_r(const Jobs<RefJob>& js, int total, unsigned long long* counters, hipStream_t s) {
    hipLaunchKernelGGL(me_forward_kernel<R>, dim3(total), dim3(256), 0, s, js, total, counters);
    return hipGetLastError();
}

hipError_t launch_me(int R, const Jobs<RefJob>& js, int total, unsigned long long* counters, hipStream_t s) {
#define RFSR_ME_CASE(r) \
    case r: return launch_me_r<r>(js, total, counters, s);
    switch (R) {
        RFSR_ME_CASE(0) RFSR_ME_CASE(1) RFSR_ME_CASE(2) RFSR_ME_CASE(3) RFSR_ME_CASE(4)
        RFSR_ME_CASE(5) RFSR_ME_CASE(6) RFSR_ME_CASE(7) RFSR_ME_CASE(8) RFSR_ME_CASE(9)
        RFSR_ME_CASE(10) RFSR_ME_CASE(11) RFSR_ME_CASE(12) RFSR_ME_CASE(13) RFSR_ME_CASE(14)
        RFSR_ME_CASE(15)
        default: return hipErrorInvalidValue;
    }
#undef RFSR_ME_CASE
}

}  // namespace

bool check_needs_windows(int check) {
    return check == RFSR_CHECK_RME || check == RFSR_CHECK_RMC || check == RFSR_CHECK_FRMC ||
           check == RFSR_CHECK_NNC_FRMC;
}

hipError_t launch_windows(const Jobs<FrameJob>& js, int total_groups, hipStream_t s) {
    if (total_groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(windows_kernel, dim3(total_groups), dim3(256), 0, s, js);
    return hipGetLastError();
}

hipError_t launch_project(const Jobs<FrameJob>& js, int total_groups, hipStream_t s) {
    if (total_groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(project_kernel, dim3(total_groups), dim3(256), 0, s, js);
    return hipGetLastError();
}

hipError_t launch_motion(const Jobs<RefJob>& js, int total_tiles, int total_px, int total_frmc,
                         const rfsr_me_params& me, unsigned long long* counters, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipError_t err = launch_me(me.search, js, total_tiles, counters, s);
    if (err != hipSuccess) return err;
    const int rr = me.rmc_radius > 0 ? me.rmc_radius : me.search;
    CheckOpts opts;
    memset(&opts, 0, sizeof(opts));
    opts.raw = me.cost_norm == 0;
    opts.nnc_raw = me.nnc_center == RFSR_NNC_RAW;
    opts.nf = me.n_frmc;
    for (int i = 0; i < me.n_frmc && i < kMaxFrmc; ++i) opts.f[i] = me.frmc[i];
    const bool custom = opts.nf > 0;
    const dim3 gpx(total_px), blk(256);
    switch (me.check) {
        case RFSR_CHECK_NONE:
            hipLaunchKernelGGL(accept_all_kernel, gpx, blk, 0, s, js, counters);
            break;
        case RFSR_CHECK_RME:
            hipLaunchKernelGGL(reverse_me_kernel, gpx, blk, 0, s, js, me.search, opts.raw, counters);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            hipLaunchKernelGGL(rme_accept_kernel, gpx, blk, 0, s, js, counters);
            break;
        case RFSR_CHECK_RMC:
            hipLaunchKernelGGL((rmc_kernel<true, false>), gpx, blk, 0, s, js, rr, opts, counters);
            break;
        case RFSR_CHECK_FRMC:
            if (custom) hipLaunchKernelGGL((rmc_kernel<false, true>), gpx, blk, 0, s, js, rr, opts, counters);
            else hipLaunchKernelGGL((rmc_kernel<false, false>), gpx, blk, 0, s, js, rr, opts, counters);
            break;
        case RFSR_CHECK_NNC:
        case RFSR_CHECK_NNC_FRMC: {
            const bool cascade = me.check == RFSR_CHECK_NNC_FRMC;
            hipLaunchKernelGGL(median_kernel, gpx, blk, 0, s, js);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            hipLaunchKernelGGL(nnc_kernel, gpx, blk, 0, s, js, opts.nnc_raw, counters, !cascade);
            if (cascade) {
                if ((err = hipGetLastError()) != hipSuccess) return err;
                if (custom)
                    hipLaunchKernelGGL(frmc_tile_kernel<true>, dim3(total_frmc), blk, 0, s, js, opts, counters);
                else
                    hipLaunchKernelGGL(frmc_tile_kernel<false>, dim3(total_frmc), blk, 0, s, js, opts, counters);
            }
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rfsr
