// Register-resident FFT building blocks of the FSR kernels (gfx950): a
// 4-point DFT, a 16-point DFT in registers and a 32-point DFT split over the
// two 32-lane halves of a wavefront.  T is double or float.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfsr {

template <typename T>
__device__ __forceinline__ void dft4(T (&r)[4], T (&i)[4]) {
    // A_k = sum_j a_j exp(-2 pi i j k / 4)
    const T t0r = r[0] + r[2], t0i = i[0] + i[2];
    const T t1r = r[0] - r[2], t1i = i[0] - i[2];
    const T t2r = r[1] + r[3], t2i = i[1] + i[3];
    const T t3r = r[1] - r[3], t3i = i[1] - i[3];
    r[0] = t0r + t2r; i[0] = t0i + t2i;
    r[2] = t0r - t2r; i[2] = t0i - t2i;
    r[1] = t1r + t3i; i[1] = t1i - t3r;   // t1 - i t3
    r[3] = t1r - t3i; i[3] = t1i + t3r;   // t1 + i t3
}

// In-register forward 16-point DFT, natural order in and out.
// u = i0 + 4 i1, k = k0 + 4 k1:  U[k] = sum_i0 w4^(i0 k1) w16^(i0 k0) sum_i1 u w4^(i1 k0).
// tw: exp(-2 pi i t / 32), t = 0..31 (re, im interleaved).
template <typename T>
__device__ __forceinline__ void fft16(T (&re)[16], T (&im)[16], const T* __restrict__ tw) {
    T tr[16], ti[16];
#pragma unroll
    for (int i0 = 0; i0 < 4; ++i0) {
        T ar[4], ai[4];
#pragma unroll
        for (int i1 = 0; i1 < 4; ++i1) { ar[i1] = re[i0 + 4 * i1]; ai[i1] = im[i0 + 4 * i1]; }
        dft4(ar, ai);
#pragma unroll
        for (int k0 = 0; k0 < 4; ++k0) {
            const int e = i0 * k0;   // w16^e = w32^(2e)
            if (e == 0) {
                tr[i0 * 4 + k0] = ar[k0]; ti[i0 * 4 + k0] = ai[k0];
            } else {
                const T cr = tw[4 * e], ci = tw[4 * e + 1];
                tr[i0 * 4 + k0] = ar[k0] * cr - ai[k0] * ci;
                ti[i0 * 4 + k0] = ar[k0] * ci + ai[k0] * cr;
            }
        }
    }
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0) {
        T br[4], bi[4];
#pragma unroll
        for (int i0 = 0; i0 < 4; ++i0) { br[i0] = tr[i0 * 4 + k0]; bi[i0] = ti[i0 * 4 + k0]; }
        dft4(br, bi);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) { re[k0 + 4 * k1] = br[k1]; im[k0 + 4 * k1] = bi[k1]; }
    }
}

// Exchange the upper 32 lanes of a with the lower 32 lanes of b (gfx950
// v_permlane32_swap, one per dword): afterwards a holds (a_lower, b_lower)
// and b holds (a_upper, b_upper) over lanes (0-31, 32-63).
__device__ __forceinline__ void swap_halves(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap_halves(double& a, double& b) {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)__double2loint(a), (uint32_t)__double2loint(b),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)__double2hiint(a), (uint32_t)__double2hiint(b),
                                                     false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// 32-point forward DFT of x[m], m = i + 16 h held by the lane pair (h=0, h=1)
// at register i.  Afterwards register k' of lane h holds X[2 k' + h].
// The radix-2 step pairs x[m] with x[m + 16]: swapping the lane halves of
// registers i and i + 8 brings x[i], x[i + 16] into the lower lanes and
// x[i + 8], x[i + 24] into the upper ones, the butterfly runs in registers,
// and the same swap puts the sums back in the lower lanes and the twiddled
// differences in the upper lanes.
template <typename T>
__device__ __forceinline__ void fft32_pair(T (&re)[16], T (&im)[16], int h, const T* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        swap_halves(re[i], re[i + 8]);
        swap_halves(im[i], im[i + 8]);
        const T ar = re[i], ai = im[i], br = re[i + 8], bi = im[i + 8];
        const T dr = ar - br, di = ai - bi;
        re[i] = ar + br;
        im[i] = ai + bi;
        // twiddle w32^i for the pair in the lower lanes, w32^(i+8) in the upper ones
        const T c0 = tw[2 * i], s0 = tw[2 * i + 1];          // uniform loads, then select
        const T c1 = tw[2 * i + 16], s1 = tw[2 * i + 17];
        const T cr = h ? c1 : c0;
        const T ci = h ? s1 : s0;
        re[i + 8] = fma(-di, ci, dr * cr);
        im[i + 8] = fma(di, cr, dr * ci);
        swap_halves(re[i], re[i + 8]);
        swap_halves(im[i], im[i + 8]);
    }
    fft16(re, im, tw);
}

}  // namespace rfsr
