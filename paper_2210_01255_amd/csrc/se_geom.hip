// se_geom.hip -- cell list: validation, grid anchors, bin keys, stable sort,
// sorted gathers and cell starts (Sec. 4.1.2 cell list; Sec. 3.3 window anchors).
//
// The sort is a least-significant-digit radix sort of (bin key, point index)
// pairs with 8-bit digits, written for this library: per pass a count kernel
// (digit histogram of each block of 4096 keys), an exclusive scan of the
// histograms in digit-major order (one workgroup), and a scatter kernel that
// ranks each key among the equal digits before it in its block (wavefront
// ballots over the digit bits, then per-wave counts in LDS).  Every position
// follows from the keys alone, so the permutation is the stable one and does
// not depend on scheduling; no pass clears memory, so binding can be recorded
// into a HIP graph.
#include <algorithm>
#include <cstring>

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

// ---------------------------------------------------------------------------
// Radix sort of (key, value) pairs.
namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;                     // keys per thread
constexpr int kRsBlock = kRsThreads * kRsItems;  // keys per block
constexpr int kRsBits = 8;
constexpr int kRsDigits = 1 << kRsBits;

__device__ __forceinline__ int rs_digit(int key, int shift, int mask) { return (key >> shift) & mask; }

// hist[d * nblocks + b] = number of keys of block b whose digit is d.
__global__ void __launch_bounds__(kRsThreads) k_rs_count(const int* __restrict__ keys, int64_t n, int shift, int mask,
                                                       int nblocks, int* __restrict__ hist)
{
    __shared__ int cnt[kRsDigits];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsBlock;
#pragma unroll 4
    for (int k = 0; k < kRsItems; k++) {
        const int64_t i = base + (int64_t)k * kRsThreads + t;
        if (i < n) atomicAdd(&cnt[rs_digit(keys[i], shift, mask)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = cnt[t];
}

// Keys of block b in their input order k * 256 + t (k = 0 .. 15): each wave
// takes 64 consecutive keys, finds the lanes holding its digit with one
// ballot per digit bit, and ranks itself among the lower lanes; the wave
// counts per digit are combined in wave order and carried over k, so that a
// key's position is off[d] + (equal digits before it in the block).
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const int* __restrict__ keys_in,
                                                         const int* __restrict__ vals_in, int64_t n, int shift,
                                                         int mask, int nbits, int nblocks,
                                                         const int* __restrict__ off, int* __restrict__ keys_out,
                                                         int* __restrict__ vals_out)
{
    constexpr int W = kRsThreads / 64;
    __shared__ int run[kRsDigits];        // position of the next key of each digit
    __shared__ int wcnt[W][kRsDigits];    // keys of each digit per wave in this step
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    run[t] = off[(int64_t)t * nblocks + blockIdx.x];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRsBlock;
    for (int k = 0; k < kRsItems; k++) {
#pragma unroll
        for (int w = 0; w < W; w++) wcnt[w][t] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)k * kRsThreads + t;
        const bool valid = i < n;
        const int key = valid ? keys_in[i] : 0;
        const int val = valid ? vals_in[i] : 0;
        const int d = rs_digit(key, shift, mask);
        uint64_t peers = __ballot(valid);
        if (!valid) peers = 0;
        for (int b = 0; b < nbits; b++) {
            const uint64_t on = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? on : ~on;
        }
        const int rank = __builtin_popcountll(peers & below);
        // the lowest lane of each group records the group's size
        if (valid && rank == 0) wcnt[wv][d] = __builtin_popcountll(peers);
        __syncthreads();
        int pre = 0;
        for (int w = 0; w < wv; w++) pre += wcnt[w][d];
        const int pos = run[d] + pre + rank;
        if (valid) {
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        int tot = 0;
#pragma unroll
        for (int w = 0; w < W; w++) tot += wcnt[w][t];
        run[t] += tot;
        // run[] is read again only after the next step's first barrier
    }
}

inline int rs_nblocks(int64_t n) { return (int)((n + kRsBlock - 1) / kRsBlock); }

}  // namespace

// Stable sort of (key, value) pairs by keys in [0, 2^end_bit): sorted keys to
// keys_out and the values in the same order to vals_out (the inputs are not
// written).  tmp holds a second pair of arrays and the digit histograms
// (se_sort_tmp_bytes).
se_status se_sort_pairs_raw(void* tmp, size_t tmp_bytes, const int* keys_in, int* keys_out, const int* vals_in,
                            int* vals_out, int64_t n, int end_bit, hipStream_t s)
{
    if (n <= 0) return SE_OK;
    if (n > ((int64_t)1 << 31) - 1 || end_bit < 1 || end_bit > 31 || tmp_bytes < se_sort_tmp_bytes(n, end_bit))
        return SE_ERR_ARG;
    const int nb = rs_nblocks(n);
    int* kt = (int*)tmp;
    int* vt = kt + n;
    int* hist = vt + n;
    const int npass = (end_bit + kRsBits - 1) / kRsBits;
    const int* ki = keys_in;
    const int* vi = vals_in;
    for (int pass = 0; pass < npass; pass++) {
        // the last pass writes the caller's arrays; earlier ones alternate so
        // that it does
        const bool to_out = ((npass - 1 - pass) % 2) == 0;
        int* ko = to_out ? keys_out : kt;
        int* vo = to_out ? vals_out : vt;
        const int shift = pass * kRsBits;
        const int nbits = std::min(kRsBits, end_bit - shift);
        const int mask = (1 << nbits) - 1;
        hipLaunchKernelGGL(k_rs_count, dim3(nb), dim3(kRsThreads), 0, s, ki, n, shift, mask, nb, hist);
        se_launch_scan_excl(hist, (int64_t)kRsDigits * nb, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kRsThreads), 0, s, ki, vi, n, shift, mask, nbits, nb, hist,
                           ko, vo);
        ki = ko;
        vi = vo;
    }
    return hipGetLastError() == hipSuccess ? SE_OK : SE_ERR_HIP;
}

size_t se_sort_tmp_bytes(int64_t n, int end_bit)
{
    (void)end_bit;
    return sizeof(int) * ((size_t)2 * (size_t)std::max<int64_t>(n, 1) + (size_t)kRsDigits * rs_nblocks(std::max<int64_t>(n, 1)) + 1);
}
