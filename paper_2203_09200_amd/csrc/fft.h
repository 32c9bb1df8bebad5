// Register-resident FFT building blocks of the FSR kernels (gfx950): a
// 4-point DFT, a 16-point DFT in registers and a 32-point DFT split over the
// two 32-lane halves of a wavefront.  T is double or float.
#pragma once

#include <hip/hip_runtime.h>

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

// 32-point forward DFT of x[m], m = i + 16 h held by the lane pair (h=0, h=1)
// at register i.  Afterwards register k' of lane h holds X[2 k' + h].
template <typename T>
__device__ __forceinline__ void fft32_pair(T (&re)[16], T (&im)[16], int h, const T* __restrict__ tw) {
    const T sgn = h ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const T pr = __shfl_xor(re[i], 32);
        const T pi = __shfl_xor(im[i], 32);
        // h = 0: x[i] + x[i+16];  h = 1: (x[i] - x[i+16]) * w32^i
        const T ur = fma(sgn, re[i], pr);
        const T ui = fma(sgn, im[i], pi);
        if (i == 0) {
            re[i] = ur;
            im[i] = ui;
        } else {
            const T twr = tw[2 * i], twi = tw[2 * i + 1];   // uniform loads, then select
            const T cr = h ? twr : T(1);
            const T ci = h ? twi : T(0);
            re[i] = ur * cr - ui * ci;
            im[i] = ur * ci + ui * cr;
        }
    }
    fft16(re, im, tw);
}

}  // namespace rfsr
