// se_geom.hip -- cell list: validation, grid anchors, bin keys, stable sort,
// sorted gathers and cell starts (Sec. 4.1.2 cell list; Sec. 3.3 window anchors).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "se_device.h"

namespace {

__global__ void k_fill_int(int* p, int v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_double(double* p, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Periodic coordinate reduced into [0, L) (the opt-in wrap); the same
// arithmetic in binning and in the sorted copies keeps the two consistent.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
    double y = x - L * floor(x / L);
    return (y >= L || y < 0.0) ? 0.0 : y;
}

// One key per point: the bin of its grid anchor.  Invalid points (non-finite
// or outside [0, L_i)) raise a flag and are binned as if at the origin.  With
// wrap, periodic coordinates are first reduced modulo L_i.
__global__ void k_bin_keys(se_grid_geom g, const double* __restrict__ xyz, int64_t n,
                           int* __restrict__ keys, int* __restrict__ idx, int* flags, int wrap)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[3];
    int bad = 0;
    for (int d = 0; d < 3; d++) {
        x[d] = xyz[3 * i + d];
        if (wrap && g.periodic[d] && isfinite(x[d])) x[d] = wrap_coord(x[d], g.L[d]);
        if (!isfinite(x[d])) bad |= SE_FLAG_NONFINITE;
        else if (!(x[d] >= 0.0 && x[d] < g.L[d])) bad |= SE_FLAG_OUT_OF_BOX;
    }
    if (bad) {
        atomicOr(flags, bad);
        x[0] = x[1] = x[2] = 0.0;
    }
    int b[3];
    for (int d = 0; d < 3; d++) b[d] = se_anchor(g, d, x[d]) / g.B[d];
    keys[i] = (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
    idx[i] = (int)i;
}

// out[d*n + s] = xyz[perm[s]][d]; invalid points are replaced by the origin.
__global__ void k_gather_sorted(const double* __restrict__ xyz, const int* __restrict__ perm,
                                int64_t n, se_grid_geom g, double* __restrict__ out, double* __restrict__ out4,
                                int sanitize, int wrap)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    double x[3];
    bool bad = false;
    for (int d = 0; d < 3; d++) {
        x[d] = xyz[3 * o + d];
        if (wrap && g.periodic[d] && isfinite(x[d])) x[d] = wrap_coord(x[d], g.L[d]);
        if (sanitize && (!isfinite(x[d]) || !(x[d] >= 0.0 && x[d] < g.L[d]))) bad = true;
        if (!sanitize && !isfinite(x[d])) x[d] = 0.0;
    }
    for (int d = 0; d < 3; d++) out[d * n + s] = bad ? 0.0 : x[d];
    if (out4) {
        double4 v;
        v.x = bad ? 0.0 : x[0];
        v.y = bad ? 0.0 : x[1];
        v.z = bad ? 0.0 : x[2];
        v.w = 0.0;
        reinterpret_cast<double4*>(out4)[s] = v;
    }
}

// start[b] = first sorted position whose key >= b (binary search), b in [0, nbins].
__global__ void k_cell_starts(const int* __restrict__ keys, int64_t n, int64_t nbins,
                              int* __restrict__ start)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbins) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    start[b] = (int)lo;
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void se_launch_fill_int(int* p, int v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    unsigned gb = grid1d(n, 256);
    if (gb > 65536) gb = 65536;
    hipLaunchKernelGGL(k_fill_int, dim3(gb), dim3(256), 0, s, p, v, n);
}

void se_launch_fill_double(double* p, double v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    unsigned gb = grid1d(n, 256);
    if (gb > 65536) gb = 65536;
    hipLaunchKernelGGL(k_fill_double, dim3(gb), dim3(256), 0, s, p, v, n);
}

void se_launch_bin_keys(const se_grid_geom& g, const double* xyz, int64_t n, int* keys, int* idx,
                        int* flags, int wrap, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin_keys, dim3(grid1d(n, 256)), dim3(256), 0, s, g, xyz, n, keys, idx, flags, wrap);
}

void se_launch_gather_sorted(const double* xyz, const int* perm, int64_t n, const se_grid_geom& g,
                             double* out_soa, double* out_aos4, int sanitize, int wrap, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_sorted, dim3(grid1d(n, 256)), dim3(256), 0, s, xyz, perm, n, g,
                       out_soa, out_aos4, sanitize, wrap);
}

void se_launch_cell_starts(const int* sorted_keys, int64_t n, int64_t nbins, int* start, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_starts, dim3(grid1d(nbins + 1, 256)), dim3(256), 0, s, sorted_keys, n,
                       nbins, start);
}

// Stable LSD radix sort of (key, index) pairs: keys in d_keys_a, indices in
// d_vals_a; sorted keys land in d_keys_b and the permutation in the caller's
// perm buffer (passed through d_vals_a -> perm by the caller).
se_status se_sort_pairs_raw(void* tmp, size_t tmp_bytes, const int* keys_in, int* keys_out,
                            const int* vals_in, int* vals_out, int64_t n, int end_bit, hipStream_t s)
{
    size_t need = tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(tmp, need, keys_in, keys_out, vals_in, vals_out,
                                             (size_t)n, 0, end_bit, s);
    return e == hipSuccess ? SE_OK : SE_ERR_HIP;
}

size_t se_sort_tmp_bytes(int64_t n, int end_bit)
{
    size_t need = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, need, (const int*)nullptr, (int*)nullptr,
                              (const int*)nullptr, (int*)nullptr, (size_t)n, 0, end_bit, (hipStream_t)0);
    return need;
}
