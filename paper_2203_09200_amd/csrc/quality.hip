// Reconstruction quality of Sec. 4 on the GPU: PSNR and mean SSIM of a
// float32 reconstruction against the uint8 ground truth, with a border of
// `border` pixels removed and the reconstruction clipped to [0, 255].
//
// SSIM (the paper cites Wang et al. 2004 for it): 11x11 Gaussian window,
// sigma 1.5, unit sum; C1 = (0.01 * 255)^2, C2 = (0.03 * 255)^2; the mean
// over every window position inside the cropped frame.  One workgroup owns a
// 16x16 tile of window positions (and of cropped pixels for the squared
// error): it stages the 26x26 input patch of both images in LDS and each
// thread forms its window's weighted moments in float64.  Per-tile partial
// sums go to the workspace and one workgroup adds them in a fixed order, so
// the result does not depend on scheduling.
#include "common.h"

namespace rfsr {

namespace {

constexpr int kQT = 16;                 // tile edge (window positions)
constexpr int kWin = 11;                // SSIM window
constexpr int kQP = kQT + kWin - 1;     // staged patch edge

__global__ __launch_bounds__(256) void quality_tile_kernel(const uint8_t* __restrict__ ref,
                                                           const float* __restrict__ test, int H, int W,
                                                           int64_t pitch, int border, int tiles_x,
                                                           double* __restrict__ partial) {
    __shared__ double s_x[kQP][kQP];
    __shared__ double s_y[kQP][kQP];
    __shared__ double s_g[kWin];
    __shared__ double s_red[2][256];
    const int tid = threadIdx.x;
    const int Hc = H - 2 * border, Wc = W - 2 * border;   // cropped frame
    const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
    const int y0 = ty * kQT, x0 = tx * kQT;               // in cropped coordinates

    if (tid < kWin) {
        const double d = tid - (kWin - 1) / 2.0;
        s_g[tid] = exp(-d * d / (2.0 * 1.5 * 1.5));
    }
    for (int e = tid; e < kQP * kQP; e += 256) {
        const int r = e / kQP, c = e - r * kQP;
        const int y = min(y0 + r, Hc - 1), x = min(x0 + c, Wc - 1);   // clamped: in bounds
        const int64_t off = (int64_t)(y + border) * pitch + (x + border);
        s_x[r][c] = (double)ref[off];
        s_y[r][c] = fmin(fmax((double)test[off], 0.0), 255.0);
    }
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int k = 0; k < kWin; ++k) sum += s_g[k];
        s_red[0][0] = sum;
    }
    __syncthreads();
    const double gnorm = 1.0 / s_red[0][0];
    __syncthreads();

    const int r = tid / kQT, c = tid - r * kQT;
    double ssim = 0.0, sq = 0.0;
    if (y0 + r < Hc && x0 + c < Wc) {
        const double d = s_x[r][c] - s_y[r][c];
        sq = d * d;
    }
    if (y0 + r <= Hc - kWin && x0 + c <= Wc - kWin) {
        double mx = 0, my = 0, mxx = 0, myy = 0, mxy = 0;
        for (int u = 0; u < kWin; ++u) {
            const double gu = s_g[u] * gnorm;
            for (int v = 0; v < kWin; ++v) {
                const double w = gu * (s_g[v] * gnorm);
                const double a = s_x[r + u][c + v], b = s_y[r + u][c + v];
                mx = fma(w, a, mx);
                my = fma(w, b, my);
                mxx = fma(w, a * a, mxx);
                myy = fma(w, b * b, myy);
                mxy = fma(w, a * b, mxy);
            }
        }
        const double C1 = (0.01 * 255.0) * (0.01 * 255.0), C2 = (0.03 * 255.0) * (0.03 * 255.0);
        const double sxx = mxx - mx * mx, syy = myy - my * my, sxy = mxy - mx * my;
        ssim = ((2.0 * mx * my + C1) * (2.0 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2));
    }
    s_red[0][tid] = ssim;
    s_red[1][tid] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            s_red[0][tid] += s_red[0][tid + s];
            s_red[1][tid] += s_red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        partial[2 * blockIdx.x] = s_red[0][0];
        partial[2 * blockIdx.x + 1] = s_red[1][0];
    }
}

__global__ __launch_bounds__(256) void quality_final_kernel(const double* __restrict__ partial, int n,
                                                            double n_px, double n_win,
                                                            double* __restrict__ result) {
    __shared__ double s_red[2][256];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < n; i += 256) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    s_red[0][tid] = a;
    s_red[1][tid] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            s_red[0][tid] += s_red[0][tid + s];
            s_red[1][tid] += s_red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double mse = s_red[1][0] / n_px;
        result[0] = 10.0 * log10(255.0 * 255.0 / mse);   // +inf for a perfect reconstruction
        result[1] = s_red[0][0] / n_win;
    }
}

}  // namespace

int quality_tiles(int H, int W, int border) {
    const int Hc = H - 2 * border, Wc = W - 2 * border;
    return ((Hc + kQT - 1) / kQT) * ((Wc + kQT - 1) / kQT);
}

hipError_t launch_quality(const uint8_t* ref, const float* test, int H, int W, int64_t pitch, int border,
                          double* partial, double* result, hipStream_t s) {
    const int Hc = H - 2 * border, Wc = W - 2 * border;
    const int tiles_x = (Wc + kQT - 1) / kQT;
    const int n = quality_tiles(H, W, border);
    hipLaunchKernelGGL(quality_tile_kernel, dim3(n), dim3(256), 0, s, ref, test, H, W, pitch, border, tiles_x,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(quality_final_kernel, dim3(1), dim3(256), 0, s, partial, n, (double)Hc * Wc,
                       (double)(Hc - kWin + 1) * (Wc - kWin + 1), result);
    return hipGetLastError();
}

}  // namespace rfsr
