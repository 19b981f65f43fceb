// se_d0.hip -- free-space (D = 0) kernel precomputation, Sec. 3.5:
//  (i)   the modified kernel Ahat_R^{0P} on the upsampled (s0 M') grid:
//        harmonic  Hhat = 4 pi/k^2 (1 - cos(R k))              eq. (vico-harmonic-0p)
//        biharmonic Bhat = -8 pi/k^4 (1 + cos(R k)/2 - 3 sin(R k)/(2 R k))
//                                                              eq. (optimal-biharmonic-0p)
//        with the limits 2 pi R^2 and -pi R^4/15 at k = 0;
//  (ii)  3-D inverse FFT to real space;
//  (iii) truncation to the (2M')^3 points around the origin, and for the
//        biharmonic the tensor-product mollifier with the (4+4)-point
//        transition band f(t) = e^{-a^2 t^2} + e^{-a^2 (t-7)^2},
//        a = (2/7) sqrt(ln 100);
//  (iv)  3-D FFT on the (2M')^3 grid -> Ahat_{R,tr}, stored as the real half
//        spectrum used by the scaling step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "se_device.h"

namespace {

// 1 + cos(x)/2 - 3 sin(x)/(2x) = sum_{n>=2} (-1)^n (n-1) x^{2n}/(2n+1)!
__device__ double bih_bracket_over_x4(double x)
{
    if (x < 1.5) {
        double x2 = x * x, term = 1.0 / 120.0, sum = 0.0;  // n = 2: 1/5!
        double pw = 1.0;                                   // x^{2n-4}
        double fact = 120.0;                               // (2n+1)!
        for (int n = 2; n <= 14; n++) {
            term = ((n & 1) ? -1.0 : 1.0) * (n - 1) * pw / fact;
            sum += term;
            pw *= x2;
            fact *= (2.0 * n + 2.0) * (2.0 * n + 3.0);
        }
        return sum;
    }
    double x4 = x * x * x * x;
    return (1.0 + 0.5 * cos(x) - 1.5 * sin(x) / x) / x4;
}

__global__ void k_d0_fill(double2* spec, int n0x, int n0y, int n0z, double hx, double hy, double hz, double R,
                          int biharmonic, double inv_vol)
{
    const int hxn = n0x / 2 + 1;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)hxn * n0y * n0z;
    if (i >= total) return;
    int ix = (int)(i % hxn);
    int iy = (int)((i / hxn) % n0y);
    int iz = (int)(i / ((int64_t)hxn * n0y));
    double kx = 2.0 * M_PI * ix / (hx * n0x);
    double ky = 2.0 * M_PI * (iy < n0y / 2 ? iy : iy - n0y) / (hy * n0y);
    double kz = 2.0 * M_PI * (iz < n0z / 2 ? iz : iz - n0z) / (hz * n0z);
    double k = sqrt(kx * kx + ky * ky + kz * kz);
    double v;
    if (biharmonic) {
        v = -8.0 * M_PI * R * R * R * R * bih_bracket_over_x4(R * k);
    } else {
        double s = sin(0.5 * R * k);
        v = (k == 0.0) ? 2.0 * M_PI * R * R : 8.0 * M_PI * s * s / (k * k);
    }
    spec[i] = make_double2(v * inv_vol, 0.0);
}

__device__ __forceinline__ double mollifier(int n, int n2)
{
    const double a2 = (4.0 / 49.0) * log(100.0);
    int t = -1;
    if (n < 4) t = 3 - n;
    else if (n >= n2 - 4) t = n - (n2 - 4);
    if (t < 0) return 1.0;
    return exp(-a2 * t * t) + exp(-a2 * (t - 7) * (t - 7));
}

// grid2[j] = A(o_j) * mu, o = signed offset of index j on the 2M' grid
__global__ void k_d0_truncate(const double* grid0, int n0x, int n0y, int n0z, double* grid2, int mx, int my,
                              int mz, int mollify)
{
    const int n2x = 2 * mx, n2y = 2 * my, n2z = 2 * mz;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)n2x * n2y * n2z;
    if (i >= total) return;
    int jx = (int)(i % n2x), jy = (int)((i / n2x) % n2y), jz = (int)(i / ((int64_t)n2x * n2y));
    int ox = jx < mx ? jx : jx - n2x, oy = jy < my ? jy : jy - n2y, oz = jz < mz ? jz : jz - n2z;
    int sx = (ox + n0x) % n0x, sy = (oy + n0y) % n0y, sz = (oz + n0z) % n0z;
    double v = grid0[((int64_t)sz * n0y + sy) * n0x + sx];
    if (mollify) v *= mollifier(ox + mx, n2x) * mollifier(oy + my, n2y) * mollifier(oz + mz, n2z);
    grid2[i] = v;
}

__global__ void k_d0_extract(const double2* spec, double* tab, int64_t n, double h3)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tab[i] = spec[i].x * h3;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

se_status se_d0_precompute(se_plan* p)
{
    const se_params& par = p->par;
    const int biharmonic = p->kernel == SE_STOKESLET || p->kernel == SE_STRESSLET;
    int n0[3], m[3], n2[3];
    double h[3];
    for (int d = 0; d < 3; d++) {
        n0[d] = par.n0_fft[d];
        m[d] = p->g.Mg[d];
        n2[d] = p->Nfft[d];
        h[d] = p->g.h[d];
    }
    const int64_t nh0 = (int64_t)(n0[0] / 2 + 1) * n0[1] * n0[2];
    const int64_t nr0 = (int64_t)n0[0] * n0[1] * n0[2];
    const int64_t nh2 = (int64_t)(n2[0] / 2 + 1) * n2[1] * n2[2];
    const int64_t nr2 = (int64_t)n2[0] * n2[1] * n2[2];
    double *spec0 = nullptr, *grid0 = nullptr, *spec2 = nullptr, *grid2 = nullptr, *tw0 = nullptr;
    std::vector<double> twh;
    int off0[4];
    se_fft_twiddles(n0, &twh, off0);
    bool ok = hipMalloc(&spec0, nh0 * 16) == hipSuccess && hipMalloc(&grid0, nr0 * 8) == hipSuccess &&
              hipMalloc(&spec2, nh2 * 16) == hipSuccess && hipMalloc(&grid2, nr2 * 8) == hipSuccess &&
              hipMalloc(&tw0, twh.size() * 8) == hipSuccess;
    se_status st = SE_OK;
    if (!ok) {
        st = SE_ERR_NOMEM;
    } else {
        if (hipMemcpy(tw0, twh.data(), twh.size() * 8, hipMemcpyHostToDevice) != hipSuccess) st = SE_ERR_HIP;
    }
    if (st == SE_OK) {
        hipStream_t s = 0;
        double vol0 = h[0] * n0[0] * h[1] * n0[1] * h[2] * n0[2];
        hipLaunchKernelGGL(k_d0_fill, dim3(blocks(nh0)), dim3(256), 0, s, (double2*)spec0, n0[0], n0[1], n0[2], h[0],
                           h[1], h[2], par.R, biharmonic, 1.0 / vol0);
        se_fft3d_f64(n0, n0, h, grid0, spec0, tw0, off0, 1, -1, s);
        if (hipGetLastError() != hipSuccess) st = SE_ERR_HIP;
        if (st == SE_OK) {
            hipLaunchKernelGGL(k_d0_truncate, dim3(blocks(nr2)), dim3(256), 0, s, grid0, n0[0], n0[1], n0[2], grid2,
                               m[0], m[1], m[2], biharmonic);
            se_fft3d_f64(n2, n2, h, grid2, spec2, p->d_tw, p->tw_off, 1, 1, s);
            if (hipGetLastError() != hipSuccess) st = SE_ERR_HIP;
        }
        if (st == SE_OK)
            hipLaunchKernelGGL(k_d0_extract, dim3(blocks(nh2)), dim3(256), 0, s, (const double2*)spec2, p->d_ktab,
                               nh2, h[0] * h[1] * h[2]);
        // the queued work must finish before the buffers are freed, whatever failed
        if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) st = SE_ERR_HIP;
    }
    if (spec0) hipFree(spec0);
    if (grid0) hipFree(grid0);
    if (spec2) hipFree(spec2);
    if (grid2) hipFree(grid2);
    if (tw0) hipFree(tw0);
    return st;
}
