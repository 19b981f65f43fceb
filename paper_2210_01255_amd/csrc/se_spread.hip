// se_spread.hip -- gridding (Sec. 3.2 step (i), eq. SE-gridding-disc) and
// gathering (step (v), eq. SE-gathering-disc) with the PKB window.
//
// Both kernels are tile-stationary: one workgroup owns a TX x TY x TZ block of
// grid points held in LDS and streams the points whose window support meets
// the block (points are visited through the cell list, anchor bins of the halo
// range).  Per point one wavefront evaluates only the weights inside the
// block (one lane per 1-D weight, PKB by Horner) and then covers the
// intersection with lanes over (x, y) and a loop over z.
//   gridding: LDS accumulation (ds_add), then one plain store per grid point
//             (every grid point belongs to exactly one block: no global atomics);
//   gathering: the block's grid values are read from LDS; each point's partial
//             sum over the block is reduced across the wavefront and added to
//             the point's FP64 accumulator with one atomic per component.
// Periodic axes wrap through unwrapped bin indices (each image shift of a
// point is visited once, so supports wider than the grid are handled too);
// free axes are clipped.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "se_device.h"

#define SE_TILE_THREADS 512
#define SE_TILE_WAVES (SE_TILE_THREADS / 64)

namespace {

struct se_tile_args {
    se_grid_geom g;
    const double* xs;   // sorted positions, SoA [3][n]
    int64_t n;
    const int* start;   // cell starts [nbins+1]
    const double* pkb;  // [P][nu+1]
    int P, nu;
    double tg_c;        // truncated Gaussian: exp(-tg_c d^2), d in grid units; 0: PKB
    int chunk;          // register-tiled kernels: candidates per work item (a multiple of the batch)
    const int* xoff;    // exclusive scan over tiles of the items beyond each tile's first [ntiles + 1]
    int ntile[3];
    void* grid;         // real grid [ncomp][Mz][My][Mx]
    const void* fs;     // sorted strengths [ncomp][n] (gridding)
    double* u;          // accumulators [3][n] (gathering)
};

template <typename R>
__device__ __forceinline__ R shfl_r(R v, int src) { return __shfl(v, src, 64); }

// Intersection of one point's window support with the block, per axis.
struct se_isect {
    int lo[3], ex[3], qoff[3];
    double t[3];
};

__device__ __forceinline__ bool point_isect(const se_grid_geom& g, const double* xp, const int* shift,
                                            const int* t0, const int* te, int P, se_isect& o)
{
    const int half = P / 2;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double u = se_gridcoord(g, d, xp[d]);
        int a = (int)floor(u);
        a = a < 0 ? 0 : (a > g.Mg[d] - 1 ? g.Mg[d] - 1 : a);
        o.t[d] = u - a;
        int au = a + shift[d];
        int first = au - half + 1;
        int l = max(t0[d], first);
        int h = min(t0[d] + te[d] - 1, au + half);
        o.lo[d] = l;
        o.ex[d] = h - l + 1;
        o.qoff[d] = l - first;
        ok = ok && (l <= h);
    }
    return ok;
}

// Bins (unwrapped) whose anchors can reach the block [t0, t0+te).
__device__ __forceinline__ void halo_bins(const se_grid_geom& g, const int* t0, const int* te, int P,
                                          int* b0, int* nbr)
{
    const int half = P / 2;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int A0 = t0[d] - half, A1 = t0[d] + te[d] - 2 + half;
        int bb0 = se_floordiv(A0, g.B[d]), bb1 = se_floordiv(A1, g.B[d]);
        if (!g.periodic[d]) {
            bb0 = max(bb0, 0);
            bb1 = min(bb1, g.nb[d] - 1);
        }
        b0[d] = bb0;
        nbr[d] = max(bb1 - bb0 + 1, 0);
    }
}

__device__ __forceinline__ int wrap_bin(const se_grid_geom& g, const int* ub, int* shift)
{
    int wb[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (g.periodic[d]) {
            int k = se_floordiv(ub[d], g.nb[d]);
            wb[d] = ub[d] - k * g.nb[d];
            shift[d] = k * g.Mg[d];
        } else {
            wb[d] = ub[d];
            shift[d] = 0;
        }
    }
    return (wb[2] * g.nb[1] + wb[1]) * g.nb[0] + wb[0];
}

__device__ __forceinline__ void tile_origin_at(int bid, const int* ntile, int TX, int TY, int TZ,
                                               const se_grid_geom& g, int* t0, int* te)
{
    int tx = bid % ntile[0];
    int ty = (bid / ntile[0]) % ntile[1];
    int tz = bid / (ntile[0] * ntile[1]);
    t0[0] = tx * TX;
    t0[1] = ty * TY;
    t0[2] = tz * TZ;
    te[0] = min(TX, g.Mg[0] - t0[0]);
    te[1] = min(TY, g.Mg[1] - t0[1]);
    te[2] = min(TZ, g.Mg[2] - t0[2]);
}

__device__ __forceinline__ void tile_origin(const int* ntile, int TX, int TY, int TZ, const se_grid_geom& g,
                                            int* t0, int* te)
{
    tile_origin_at(se_xcd_block(blockIdx.x, gridDim.x), ntile, TX, TY, TZ, g, t0, te);
}

// Unrolled Horner with SE_MAX_NU + 1 coefficients (zero padded beyond nu,
// which leaves the arithmetic of the lower-degree polynomial unchanged).
template <typename R>
__device__ __forceinline__ R pkb_weight(const double* coef, int q, R s)
{
    const double* c = coef + q * (SE_MAX_NU + 1);
    R sig = (R)2 * s - (R)1;
    R acc = (R)c[SE_MAX_NU];
#pragma unroll
    for (int k = SE_MAX_NU - 1; k >= 0; k--) acc = acc * sig + (R)c[k];
    return acc;
}

// Weight of grid offset q (0 .. P-1) for a point at fractional position t in
// its anchor cell, given s = 1 - t: the PKB polynomial of subinterval q at s,
// or the truncated Gaussian at distance d = q - P/2 + s grid spacings
// (|d| <= P/2 there, so the support test is implied).
template <typename R>
__device__ __forceinline__ R win_weight(const double* coef, double tg_c, int P, int q, R s)
{
    if (tg_c > 0.0) {
        const R d = (R)(q - P / 2) + s;
        return exp(-(R)tg_c * d * d);
    }
    return pkb_weight<R>(coef, q, s);
}

__device__ __forceinline__ int rl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Per-wave walk over the points whose anchors lie in the block's halo: rows
// of bins (by, bz) are split into runs of consecutive x bins with one wrap
// shift, each run is a contiguous range of sorted points.  Points are loaded
// 64 at a time (one per lane), intersected lane-parallel, and the non-empty
// ones are handed to `body` one by one (uniform control flow).
template <typename Body>
__device__ __forceinline__ void walk_points(const se_tile_args& a, const int* t0, const int* te, int wave, int lane,
                                            Body&& body)
{
    const se_grid_geom& g = a.g;
    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int nrows = nbr[1] * nbr[2];
    const int64_t n = a.n;
    for (int row = wave; row < nrows; row += SE_TILE_WAVES) {
        int uy = b0[1] + row % nbr[1], uz = b0[2] + row / nbr[1];
        int sy = 0, sz = 0, wy = uy, wz = uz;
        if (g.periodic[1]) {
            int k = se_floordiv(uy, g.nb[1]);
            wy = uy - k * g.nb[1];
            sy = k * g.Mg[1];
        }
        if (g.periodic[2]) {
            int k = se_floordiv(uz, g.nb[2]);
            wz = uz - k * g.nb[2];
            sz = k * g.Mg[2];
        }
        const int rowbase = (wz * g.nb[1] + wy) * g.nb[0];
        int ux = b0[0];
        const int uxe = b0[0] + nbr[0] - 1;
        while (ux <= uxe) {
            int kx = g.periodic[0] ? se_floordiv(ux, g.nb[0]) : 0;
            int wx0 = ux - kx * g.nb[0];
            int run = min(uxe - ux + 1, g.nb[0] - wx0);
            int shift[3] = {kx * g.Mg[0], sy, sz};
            int s_beg = a.start[rowbase + wx0], s_end = a.start[rowbase + wx0 + run];
            for (int base = s_beg; base < s_end; base += 64) {
                int s = base + lane;
                bool valid = s < s_end;
                int sc = valid ? s : s_beg;
                double xp[3] = {a.xs[sc], a.xs[n + sc], a.xs[2 * n + sc]};
                se_isect q;
                bool ok = point_isect(g, xp, shift, t0, te, a.P, q) && valid;
                uint64_t mask = __ballot(ok);
                body(mask, sc, q);
            }
            ux += run;
        }
    }
}

template <typename R, int NC, int TX, int TY, int TZ>
__global__ void __launch_bounds__(SE_TILE_THREADS) k_spread(se_tile_args a)
{
    extern __shared__ double smem_d[];
    constexpr int TV = TX * TY * TZ;
    double* s_pkb = smem_d;
    R* acc = (R*)(smem_d + SE_MAX_P * (SE_MAX_NU + 1));
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin(a.ntile, TX, TY, TZ, g, t0, te);
    for (int i = tid; i < NC * TV; i += SE_TILE_THREADS) acc[i] = (R)0;
    for (int i = tid; i < SE_MAX_P * (SE_MAX_NU + 1); i += SE_TILE_THREADS) {
        int q = i / (SE_MAX_NU + 1), k = i - q * (SE_MAX_NU + 1);
        s_pkb[i] = (q < a.P && k <= a.nu) ? a.pkb[q * (a.nu + 1) + k] : 0.0;
    }
    __syncthreads();
    const R* fs = (const R*)a.fs;
    const int64_t n = a.n;
    walk_points(a, t0, te, wave, lane, [&](uint64_t mask, int sc, const se_isect& q) {
        R fl[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) fl[c] = fs[c * n + sc];
        while (mask) {
            const int j = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int lo0 = rl_i(q.lo[0], j), lo1 = rl_i(q.lo[1], j), lo2 = rl_i(q.lo[2], j);
            const int ex0 = rl_i(q.ex[0], j), ex1 = rl_i(q.ex[1], j), ex2 = rl_i(q.ex[2], j);
            const int qo0 = rl_i(q.qoff[0], j), qo1 = rl_i(q.qoff[1], j), qo2 = rl_i(q.qoff[2], j);
            R f[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) f[c] = se_readlane(fl[c], j);
            int dim, qq;
            double tt;
            if (lane < ex0) {
                dim = 0;
                qq = qo0 + lane;
            } else if (lane < ex0 + ex1) {
                dim = 1;
                qq = qo1 + lane - ex0;
            } else {
                dim = 2;
                qq = qo2 + min(lane - ex0 - ex1, ex2 - 1);
            }
            const double tj0 = se_readlane(q.t[0], j), tj1 = se_readlane(q.t[1], j), tj2 = se_readlane(q.t[2], j);
            tt = dim == 0 ? tj0 : (dim == 1 ? tj1 : tj2);
            const R w = win_weight<R>(s_pkb, a.tg_c, a.P, qq, (R)(1.0 - tt));
            const int nxy = ex0 * ex1;
            const int zl = lo2 - t0[2], yl = lo1 - t0[1], xl = lo0 - t0[0];
            for (int base = 0; base < nxy; base += 64) {
                int idx = base + lane;
                bool act = idx < nxy;
                int idc = act ? idx : 0;
                int iy = idc / ex0;
                int ix = idc - iy * ex0;
                R wx = shfl_r(w, ix);
                R wy = shfl_r(w, ex0 + iy);
                R gv[NC];
#pragma unroll
                for (int c = 0; c < NC; c++) gv[c] = wx * wy * f[c];
                int lb = (zl * TY + yl + iy) * TX + xl + ix;
                for (int iz = 0; iz < ex2; iz++) {
                    R wz = se_readlane(w, ex0 + ex1 + iz);
                    if (act) {
#pragma unroll
                        for (int c = 0; c < NC; c++) atomicAdd(&acc[c * TV + lb + iz * TX * TY], wz * gv[c]);
                    }
                }
            }
        }
    });
    __syncthreads();
    R* grid = (R*)a.grid;
    const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
    const int64_t vol = plane * g.Mg[2];
    for (int i = tid; i < TV; i += SE_TILE_THREADS) {
        int ix = i % TX, iy = (i / TX) % TY, iz = i / (TX * TY);
        if (ix < te[0] && iy < te[1] && iz < te[2]) {
            int64_t o = (int64_t)(t0[2] + iz) * plane + (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix;
#pragma unroll
            for (int c = 0; c < NC; c++) grid[c * vol + o] = acc[c * TV + i];
        }
    }
}

template <typename R, int TX, int TY, int TZ>
__global__ void __launch_bounds__(SE_TILE_THREADS) k_gather(se_tile_args a)
{
    extern __shared__ double smem_d[];
    constexpr int TV = TX * TY * TZ;
    double* s_pkb = smem_d;
    R* tile = (R*)(smem_d + SE_MAX_P * (SE_MAX_NU + 1));
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin(a.ntile, TX, TY, TZ, g, t0, te);
    const R* grid = (const R*)a.grid;
    const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
    const int64_t vol = plane * g.Mg[2];
    for (int i = tid; i < TV; i += SE_TILE_THREADS) {
        int ix = i % TX, iy = (i / TX) % TY, iz = i / (TX * TY);
        bool in = ix < te[0] && iy < te[1] && iz < te[2];
        int64_t o = (int64_t)(t0[2] + iz) * plane + (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix;
#pragma unroll
        for (int c = 0; c < 3; c++) tile[c * TV + i] = in ? grid[c * vol + o] : (R)0;
    }
    for (int i = tid; i < SE_MAX_P * (SE_MAX_NU + 1); i += SE_TILE_THREADS) {
        int q = i / (SE_MAX_NU + 1), k = i - q * (SE_MAX_NU + 1);
        s_pkb[i] = (q < a.P && k <= a.nu) ? a.pkb[q * (a.nu + 1) + k] : 0.0;
    }
    __syncthreads();
    const int64_t n = a.n;
    walk_points(a, t0, te, wave, lane, [&](uint64_t mask, int sc, const se_isect& q) {
        const uint64_t own = mask;
        double my0 = 0.0, my1 = 0.0, my2 = 0.0;
        while (mask) {
            const int j = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int lo0 = rl_i(q.lo[0], j), lo1 = rl_i(q.lo[1], j), lo2 = rl_i(q.lo[2], j);
            const int ex0 = rl_i(q.ex[0], j), ex1 = rl_i(q.ex[1], j), ex2 = rl_i(q.ex[2], j);
            const int qo0 = rl_i(q.qoff[0], j), qo1 = rl_i(q.qoff[1], j), qo2 = rl_i(q.qoff[2], j);
            int dim, qq;
            if (lane < ex0) {
                dim = 0;
                qq = qo0 + lane;
            } else if (lane < ex0 + ex1) {
                dim = 1;
                qq = qo1 + lane - ex0;
            } else {
                dim = 2;
                qq = qo2 + min(lane - ex0 - ex1, ex2 - 1);
            }
            const double tj0 = se_readlane(q.t[0], j), tj1 = se_readlane(q.t[1], j), tj2 = se_readlane(q.t[2], j);
            const double tt = dim == 0 ? tj0 : (dim == 1 ? tj1 : tj2);
            const R w = win_weight<R>(s_pkb, a.tg_c, a.P, qq, (R)(1.0 - tt));
            const int nxy = ex0 * ex1;
            const int zl = lo2 - t0[2], yl = lo1 - t0[1], xl = lo0 - t0[0];
            R acc0 = 0, acc1 = 0, acc2 = 0;
            for (int base = 0; base < nxy; base += 64) {
                int idx = base + lane;
                bool act = idx < nxy;
                int idc = act ? idx : 0;
                int iy = idc / ex0;
                int ix = idc - iy * ex0;
                R wx = shfl_r(w, ix);
                R wy = shfl_r(w, ex0 + iy);
                R wxy = act ? wx * wy : (R)0;
                int lb = (zl * TY + yl + iy) * TX + xl + ix;
                for (int iz = 0; iz < ex2; iz++) {
                    R wz = se_readlane(w, ex0 + ex1 + iz) * wxy;
                    int o = lb + iz * TX * TY;
                    acc0 += wz * tile[o];
                    acc1 += wz * tile[TV + o];
                    acc2 += wz * tile[2 * TV + o];
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                acc0 += __shfl_xor(acc0, off, 64);
                acc1 += __shfl_xor(acc1, off, 64);
                acc2 += __shfl_xor(acc2, off, 64);
            }
            if (lane == j) {
                my0 = (double)acc0;
                my1 = (double)acc1;
                my2 = (double)acc2;
            }
        }
        if ((own >> lane) & 1ull) {
            atomicAdd(&a.u[sc], my0);
            atomicAdd(&a.u[n + sc], my1);
            atomicAdd(&a.u[2 * n + sc], my2);
        }
    });
}

// ---------------------------------------------------------------------------
// Register-tiled gridding and gathering.
// A workgroup (4 waves) owns a 16 x 16 x 8 block of grid points; wave w owns
// the 8 x 8 (x, y) columns at ((w & 1) 8, (w >> 1) 8) and keeps their 8 z
// values of every component in registers, so gridding needs no atomics at
// all and gathering reads the grid once per block.  The candidate points
// (anchors in the halo bins) are enumerated as runs of the sorted order and
// processed in batches of 64: the batch's 1-D weights restricted to the block
// (16 + 16 + 8 per point, PKB by Horner) are evaluated once into LDS, then
// every wave applies each point whose support meets its columns.
#define SE_RT_THREADS 256
#define SE_RT_KB 64
#define SE_RT_MAXSLOTS 512
#define SE_RT_TX 16
#define SE_RT_TY 16
#define SE_RT_TZ 8
#define SE_RT_NW (SE_RT_TX + SE_RT_TY + SE_RT_TZ)

template <typename R, int NC, bool GATHER>
struct se_rt_lds {
    double pkb[SE_MAX_P * (SE_MAX_NU + 1)];
    int run_beg[SE_RT_MAXSLOTS];
    int run_pre[SE_RT_MAXSLOTS + 1];
    int run_shift[SE_RT_MAXSLOTS][3];
    R w[SE_RT_KB][SE_RT_NW];
    double t[SE_RT_KB][3];
    int o[SE_RT_KB][3];
    int idx[SE_RT_KB];
    int list[4][SE_RT_KB];   // per wave: the batch's points whose support meets its columns
    int cnt[4];
    R f[GATHER ? 1 : SE_RT_KB][NC];       // gridding: the batch's strengths
    double u[GATHER ? SE_RT_KB : 1][NC];  // gathering: the batch's block partial sums
};

// Runs of sorted points whose anchor bins lie in the block's halo: one slot
// per (bin row, periodic x segment).  Returns the number of candidates.
template <typename L>
__device__ int rt_build_runs(const se_tile_args& a, const int* t0, const int* te, L& s, int tid)
{
    const se_grid_geom& g = a.g;
    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int nrows = nbr[1] * nbr[2];
    int kx0 = 0, kx1 = 0;
    if (g.periodic[0]) {
        kx0 = se_floordiv(b0[0], g.nb[0]);
        kx1 = se_floordiv(b0[0] + nbr[0] - 1, g.nb[0]);
    }
    const int nseg = nbr[0] > 0 ? kx1 - kx0 + 1 : 0;
    const int nslots = nrows * nseg;
    for (int slot = tid; slot < nslots; slot += SE_RT_THREADS) {
        const int row = slot / nseg, k = kx0 + slot % nseg;
        const int uy = b0[1] + row % nbr[1], uz = b0[2] + row / nbr[1];
        int sy = 0, sz = 0, wy = uy, wz = uz;
        if (g.periodic[1]) {
            int kk = se_floordiv(uy, g.nb[1]);
            wy = uy - kk * g.nb[1];
            sy = kk * g.Mg[1];
        }
        if (g.periodic[2]) {
            int kk = se_floordiv(uz, g.nb[2]);
            wz = uz - kk * g.nb[2];
            sz = kk * g.Mg[2];
        }
        int lo = b0[0], hi = b0[0] + nbr[0] - 1;
        if (g.periodic[0]) {
            lo = max(lo, k * g.nb[0]);
            hi = min(hi, (k + 1) * g.nb[0] - 1);
        }
        const int wx0 = lo - k * g.nb[0];
        const int rowbase = (wz * g.nb[1] + wy) * g.nb[0];
        const int beg = a.start[rowbase + wx0], end = a.start[rowbase + wx0 + (hi - lo + 1)];
        s.run_beg[slot] = beg;
        s.run_pre[slot + 1] = end - beg;  // lengths, scanned below
        s.run_shift[slot][0] = g.periodic[0] ? k * g.Mg[0] : 0;
        s.run_shift[slot][1] = sy;
        s.run_shift[slot][2] = sz;
    }
    __syncthreads();
    if (tid < 64) {
        // inclusive scan of the lengths by one wave: chunks per lane, then lanes
        const int per = (nslots + 63) / 64;
        const int c0 = tid * per, c1 = min(c0 + per, nslots);
        int sum = 0;
        for (int i = c0; i < c1; i++) sum += s.run_pre[i + 1];
        int incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int v = __shfl_up(incl, off, 64);
            if (tid >= off) incl += v;
        }
        int run = incl - sum;
        for (int i = c0; i < c1; i++) {
            run += s.run_pre[i + 1];
            s.run_pre[i + 1] = run;
        }
        if (tid == 0) s.run_pre[0] = 0;
    }
    __syncthreads();
    return nslots > 0 ? s.run_pre[nslots] : 0;
}

__device__ __forceinline__ bool rt_meets(const int* o, int P, int wxo, int wyo)
{
    return o[0] < wxo + 8 && o[0] + P > wxo && o[1] < wyo + 8 && o[1] + P > wyo && o[2] < SE_RT_TZ && o[2] + P > 0;
}

// One batch: locate candidates base .. base + KB - 1, anchor them, list them
// per wave (the points whose support meets the wave's 8 x 8 x 8 columns) and
// stage the block-restricted 1-D weights (PKB, or the truncated Gaussian
// when TG: a template parameter, so that the PKB kernels carry no second
// weight path).  Returns the batch size.
template <typename R, bool GATHER, int NC, bool TG, typename L>
__device__ int rt_stage_batch(const se_tile_args& a, const int* t0, int nslots, int total, int base, L& s, int tid)
{
    const se_grid_geom& g = a.g;
    const int nb = min(SE_RT_KB, total - base);
    if (tid < SE_RT_KB) {
        int sidx = -1;
        if (tid < nb) {
            const int f = base + tid;
            int lo = 0, hi = nslots;  // largest r with run_pre[r] <= f
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (s.run_pre[mid] <= f) lo = mid;
                else hi = mid;
            }
            sidx = s.run_beg[lo] + (f - s.run_pre[lo]);
            const int64_t n = a.n;
            const double xp[3] = {a.xs[sidx], a.xs[n + sidx], a.xs[2 * n + sidx]};
#pragma unroll
            for (int d = 0; d < 3; d++) {
                double u = se_gridcoord(g, d, xp[d]);
                int an = (int)floor(u);
                an = an < 0 ? 0 : (an > g.Mg[d] - 1 ? g.Mg[d] - 1 : an);
                s.t[tid][d] = u - an;
                s.o[tid][d] = an + s.run_shift[lo][d] - a.P / 2 + 1 - t0[d];
            }
            if constexpr (!GATHER) {
                const R* fs = (const R*)a.fs;
#pragma unroll
                for (int c = 0; c < NC; c++) s.f[tid][c] = fs[c * n + sidx];
            }
        }
        if constexpr (GATHER) {
#pragma unroll
            for (int c = 0; c < NC; c++) s.u[tid][c] = 0.0;
        }
        // one wave: ballot per sub-block, compacted lists
        int o[3] = {s.o[tid][0], s.o[tid][1], s.o[tid][2]};
        bool any = false;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            const bool m = sidx >= 0 && rt_meets(o, a.P, (w & 1) * 8, (w >> 1) * 8);
            any = any || m;
            const uint64_t bal = __ballot(m);
            const int pos = __builtin_popcountll(bal & ((1ull << tid) - 1ull));
            if (m) s.list[w][pos] = tid;
            if (tid == 0) s.cnt[w] = __builtin_popcountll(bal);
        }
        s.idx[tid] = any ? sidx : -1;  // -1: no weights needed
    }
    __syncthreads();
    for (int i = tid; i < nb * SE_RT_NW; i += SE_RT_THREADS) {
        const int p = i / SE_RT_NW, j = i - p * SE_RT_NW;
        const int dim = j < SE_RT_TX ? 0 : (j < SE_RT_TX + SE_RT_TY ? 1 : 2);
        const int coord = dim == 0 ? j : (dim == 1 ? j - SE_RT_TX : j - SE_RT_TX - SE_RT_TY);
        const int q = coord - s.o[p][dim];
        R w = (R)0;
        if (q >= 0 && q < a.P && s.idx[p] >= 0) {
            const R sl = (R)(1.0 - s.t[p][dim]);
            if constexpr (TG) {
                const R d = (R)(q - a.P / 2) + sl;
                w = exp(-(R)a.tg_c * d * d);
            } else {
                w = pkb_weight<R>(s.pkb, q, sl);
            }
        }
        s.w[p][j] = w;
    }
    __syncthreads();
    return nb;
}

// Gridding of one tile from its candidates c_lo .. c_hi - 1 (a work item).
// The first item of a tile stores its sums; further items of a crowded tile
// (EXTRA, launched after the first items) add theirs atomically.
template <typename R, int NC, bool TG, bool EXTRA>
__device__ __forceinline__ void spread_rt_tile(const se_tile_args& a, se_rt_lds<R, NC, false>& s, int tile, int c_lo,
                                               int c_hi)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin_at(tile, a.ntile, SE_RT_TX, SE_RT_TY, SE_RT_TZ, g, t0, te);
    for (int i = tid; i < SE_MAX_P * (SE_MAX_NU + 1); i += SE_RT_THREADS) {
        int q = i / (SE_MAX_NU + 1), k = i - q * (SE_MAX_NU + 1);
        s.pkb[i] = (q < a.P && k <= a.nu) ? a.pkb[q * (a.nu + 1) + k] : 0.0;
    }
    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int total = min(rt_build_runs(a, t0, te, s, tid), c_hi);
    int nseg = 1;
    if (g.periodic[0]) nseg = se_floordiv(b0[0] + nbr[0] - 1, g.nb[0]) - se_floordiv(b0[0], g.nb[0]) + 1;
    const int nslots = nbr[0] > 0 ? nbr[1] * nbr[2] * nseg : 0;
    const int wxo = (wave & 1) * 8, wyo = (wave >> 1) * 8;
    const int lx = lane & 7, ly = lane >> 3;
    R acc[SE_RT_TZ][NC];
#pragma unroll
    for (int z = 0; z < SE_RT_TZ; z++)
#pragma unroll
        for (int c = 0; c < NC; c++) acc[z][c] = (R)0;
    for (int base = c_lo; base < total; base += SE_RT_KB) {
        (void)rt_stage_batch<R, false, NC, TG>(a, t0, nslots, total, base, s, tid);
        const int cnt = __builtin_amdgcn_readfirstlane(s.cnt[wave]);
        if constexpr (NC < 6) {
            // two points per step so that the LDS reads of the second overlap
            // the arithmetic of the first
            int i = 0;
            for (; i + 1 < cnt; i += 2) {
                const int pa = __builtin_amdgcn_readfirstlane(s.list[wave][i]);
                const int pb = __builtin_amdgcn_readfirstlane(s.list[wave][i + 1]);
                const R wa = s.w[pa][wxo + lx] * s.w[pa][SE_RT_TX + wyo + ly];
                const R wb = s.w[pb][wxo + lx] * s.w[pb][SE_RT_TX + wyo + ly];
                R ga[NC], gb[NC], za[SE_RT_TZ], zb[SE_RT_TZ];
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    ga[c] = wa * s.f[pa][c];
                    gb[c] = wb * s.f[pb][c];
                }
#pragma unroll
                for (int z = 0; z < SE_RT_TZ; z++) {
                    za[z] = s.w[pa][SE_RT_TX + SE_RT_TY + z];
                    zb[z] = s.w[pb][SE_RT_TX + SE_RT_TY + z];
                }
#pragma unroll
                for (int z = 0; z < SE_RT_TZ; z++)
#pragma unroll
                    for (int c = 0; c < NC; c++) {
                        acc[z][c] += ga[c] * za[z];
                        acc[z][c] += gb[c] * zb[z];
                    }
            }
            if (i < cnt) {
                const int p = __builtin_amdgcn_readfirstlane(s.list[wave][i]);
                const R wxy = s.w[p][wxo + lx] * s.w[p][SE_RT_TX + wyo + ly];
                R gv[NC];
#pragma unroll
                for (int c = 0; c < NC; c++) gv[c] = wxy * s.f[p][c];
#pragma unroll
                for (int z = 0; z < SE_RT_TZ; z++) {
                    const R wz = s.w[p][SE_RT_TX + SE_RT_TY + z];
#pragma unroll
                    for (int c = 0; c < NC; c++) acc[z][c] += gv[c] * wz;
                }
            }
        } else {
            // six components: per point, only the pairs of z planes its
            // support meets (a wave-uniform test); the others add zero weights
            for (int i = 0; i < cnt; i++) {
                const int p = __builtin_amdgcn_readfirstlane(s.list[wave][i]);
                const int oz = __builtin_amdgcn_readfirstlane(s.o[p][2]);
                const R wxy = s.w[p][wxo + lx] * s.w[p][SE_RT_TX + wyo + ly];
                R gv[NC];
#pragma unroll
                for (int c = 0; c < NC; c++) gv[c] = wxy * s.f[p][c];
#pragma unroll
                for (int q = 0; q < SE_RT_TZ / 2; q++) {
                    if (oz < 2 * q + 2 && oz + a.P > 2 * q) {
#pragma unroll
                        for (int z = 2 * q; z < 2 * q + 2; z++) {
                            const R wz = s.w[p][SE_RT_TX + SE_RT_TY + z];
#pragma unroll
                            for (int c = 0; c < NC; c++) acc[z][c] += gv[c] * wz;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    R* grid = (R*)a.grid;
    const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
    const int64_t vol = plane * g.Mg[2];
    const int ix = wxo + lx, iy = wyo + ly;
    if (ix < te[0] && iy < te[1]) {
        const int64_t col = (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix;
#pragma unroll
        for (int z = 0; z < SE_RT_TZ; z++) {
            if (z < te[2]) {
                const int64_t o = (int64_t)(t0[2] + z) * plane + col;
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    if constexpr (EXTRA) {
                        if (acc[z][c] != (R)0) atomicAdd(&grid[c * vol + o], acc[z][c]);
                    } else {
                        grid[c * vol + o] = acc[z][c];
                    }
                }
            }
        }
    }
}

// The item -> tile map of the further items: the last tile whose offset is
// <= e (tiles without further items share their offset with the next).
__device__ __forceinline__ int rt_extra_tile(const int* xoff, int ntiles, int e)
{
    int lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (xoff[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// first item of every tile (XCD-aware tile order)
template <typename R, int NC, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 4) k_spread_rt(se_tile_args a)
{
    __shared__ se_rt_lds<R, NC, false> s;
    spread_rt_tile<R, NC, TG, false>(a, s, se_xcd_block(blockIdx.x, gridDim.x), 0, a.chunk);
}

// further items of crowded tiles; the workgroups stride through them
template <typename R, int NC, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 4) k_spread_rt_extra(se_tile_args a, int ntiles)
{
    __shared__ se_rt_lds<R, NC, false> s;
    const int items = a.xoff[ntiles];
    for (int e = blockIdx.x; e < items; e += gridDim.x) {
        const int tile = rt_extra_tile(a.xoff, ntiles, e);
        const int c0 = (1 + e - a.xoff[tile]) * a.chunk;
        spread_rt_tile<R, NC, TG, true>(a, s, tile, c0, c0 + a.chunk);
        __syncthreads();
    }
}

// Cross-lane steps of the gathering reduce-scatter, on the VALU (gfx950
// lane swaps and DPP), one helper per 32-bit width.
//   sum32(a, b): lanes 0-31 get a[l] + a[l + 32], lanes 32-63 get b[l - 32] + b[l]
//   sum16(a, b): even rows get a[l] + a[l + 16], odd rows get b[l - 16] + b[l]
__device__ __forceinline__ float rt_sum32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double rt_sum32(double a, double b)
{
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float rt_sum16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double rt_sum16(double a, double b)
{
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
// v from lane (l + 8) mod 16 (= l ^ 8) / row_half_mirror / quad_perm swaps
template <int CTRL>
__device__ __forceinline__ float rt_dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double rt_dpp(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppRor8 = 0x128, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

// Gathering of one tile to its candidates c_lo .. c_hi - 1 (a work item);
// every item adds to the targets atomically.
template <typename R, int NCG, bool TG>
__device__ __forceinline__ void gather_rt_tile(const se_tile_args& a, se_rt_lds<R, NCG, true>& s, int tile, int c_lo,
                                               int c_hi)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin_at(tile, a.ntile, SE_RT_TX, SE_RT_TY, SE_RT_TZ, g, t0, te);
    for (int i = tid; i < SE_MAX_P * (SE_MAX_NU + 1); i += SE_RT_THREADS) {
        int q = i / (SE_MAX_NU + 1), k = i - q * (SE_MAX_NU + 1);
        s.pkb[i] = (q < a.P && k <= a.nu) ? a.pkb[q * (a.nu + 1) + k] : 0.0;
    }
    const int wxo = (wave & 1) * 8, wyo = (wave >> 1) * 8;
    const int lx = lane & 7, ly = lane >> 3;
    R F[SE_RT_TZ][NCG];
    {
        const R* grid = (const R*)a.grid;
        const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
        const int64_t vol = plane * g.Mg[2];
        const int ix = wxo + lx, iy = wyo + ly;
        const bool in = ix < te[0] && iy < te[1];
        const int64_t col = in ? (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix : 0;
#pragma unroll
        for (int z = 0; z < SE_RT_TZ; z++) {
            const bool inz = in && z < te[2];
            const int64_t o = inz ? (int64_t)(t0[2] + z) * plane + col : 0;
#pragma unroll
            for (int c = 0; c < NCG; c++) F[z][c] = inz ? grid[c * vol + o] : (R)0;
        }
    }
    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int total = min(rt_build_runs(a, t0, te, s, tid), c_hi);
    int nseg = 1;
    if (g.periodic[0]) nseg = se_floordiv(b0[0] + nbr[0] - 1, g.nb[0]) - se_floordiv(b0[0], g.nb[0]) + 1;
    const int nslots = nbr[0] > 0 ? nbr[1] * nbr[2] * nseg : 0;
    const int64_t n = a.n;
    constexpr int GP = 24 / NCG;  // points per reduce-scatter group
    for (int base = c_lo; base < total; base += SE_RT_KB) {
        const int nb = rt_stage_batch<R, true, NCG, TG>(a, t0, nslots, total, base, s, tid);
        // Groups of GP points: per-lane partial sums v[NCG j + c] (24 values),
        // then one reduce-scatter over the wave: halving steps across lane
        // bits 5, 4, 3 leave lane group k (bits 5..3) with values 3k .. 3k+2,
        // and the sum over bits 2..0 completes them.
        const int cnt = __builtin_amdgcn_readfirstlane(s.cnt[wave]);
        for (int i0 = 0; i0 < cnt; i0 += GP) {
            R v[24];
#pragma unroll
            for (int j = 0; j < GP; j++) {
#pragma unroll
                for (int c = 0; c < NCG; c++) v[NCG * j + c] = (R)0;
                if (i0 + j >= cnt) continue;
                const int p = __builtin_amdgcn_readfirstlane(s.list[wave][i0 + j]);
                const R wxy = s.w[p][wxo + lx] * s.w[p][SE_RT_TX + wyo + ly];
                R acc[NCG];
#pragma unroll
                for (int c = 0; c < NCG; c++) acc[c] = (R)0;
#pragma unroll
                for (int z = 0; z < SE_RT_TZ; z++) {
                    const R wz = s.w[p][SE_RT_TX + SE_RT_TY + z];
#pragma unroll
                    for (int c = 0; c < NCG; c++) acc[c] += wz * F[z][c];
                }
#pragma unroll
                for (int c = 0; c < NCG; c++) v[NCG * j + c] = acc[c] * wxy;
            }
            const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
            R v12[12];
#pragma unroll
            for (int i = 0; i < 12; i++) v12[i] = rt_sum32(v[i], v[12 + i]);
            R v6[6];
#pragma unroll
            for (int i = 0; i < 6; i++) v6[i] = rt_sum16(v12[i], v12[6 + i]);
            R v3[3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const R mine = b3 ? v6[3 + i] : v6[i], oth = b3 ? v6[i] : v6[3 + i];
                v3[i] = mine + rt_dpp<kDppRor8>(oth);
            }
#pragma unroll
            for (int i = 0; i < 3; i++) {
                v3[i] += rt_dpp<kDppHalfMirror>(v3[i]);
                v3[i] += rt_dpp<kDppXor2>(v3[i]);
                v3[i] += rt_dpp<kDppXor1>(v3[i]);
            }
            if ((lane & 7) == 0) {
                const int grp = (b5 ? 4 : 0) + (b4 ? 2 : 0) + (b3 ? 1 : 0);
                const int k = i0 + (3 * grp) / NCG, c0 = (3 * grp) % NCG;
                if (k < cnt) {
                    const int p = s.list[wave][k];
                    atomicAdd(&s.u[p][c0], (double)v3[0]);
                    atomicAdd(&s.u[p][c0 + 1], (double)v3[1]);
                    atomicAdd(&s.u[p][c0 + 2], (double)v3[2]);
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < NCG * nb; i += SE_RT_THREADS) {
            const int p = i / NCG, c = i - NCG * p;
            const double v = s.u[p][c];
            if (v != 0.0) atomicAdd(&a.u[c * n + s.idx[p]], v);
        }
        __syncthreads();
    }
}

template <typename R, int NCG, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 3) k_gather_rt(se_tile_args a)
{
    __shared__ se_rt_lds<R, NCG, true> s;
    gather_rt_tile<R, NCG, TG>(a, s, se_xcd_block(blockIdx.x, gridDim.x), 0, a.chunk);
}

template <typename R, int NCG, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 3) k_gather_rt_extra(se_tile_args a, int ntiles)
{
    __shared__ se_rt_lds<R, NCG, true> s;
    const int items = a.xoff[ntiles];
    for (int e = blockIdx.x; e < items; e += gridDim.x) {
        const int tile = rt_extra_tile(a.xoff, ntiles, e);
        const int c0 = (1 + e - a.xoff[tile]) * a.chunk;
        gather_rt_tile<R, NCG, TG>(a, s, tile, c0, c0 + a.chunk);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Merged launches over the tiles of many plans (batches of systems): job j's
// argument record is av[j]; its first items are the workgroups boff[j] ..
// boff[j+1] - 1 (XCD-aware order over the whole launch), and its further
// items follow the device-side counts of every job.
#define SE_MULTI_MAX SE_JOB_MAX

__device__ __forceinline__ int job_of(const int* __restrict__ boff, int n, int g)
{
    int lo = 0, hi = n;  // largest j with boff[j] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// pre[j] = further items of jobs 0 .. j-1 (each job's count is the total of
// its exclusive scan over tiles)
__device__ __forceinline__ void extra_prefix(const se_tile_args* __restrict__ av, int n, int* pre)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const se_tile_args& a = av[j];
        pre[j + 1] = a.xoff[a.ntile[0] * a.ntile[1] * a.ntile[2]];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int j = 0; j < n; j++) pre[j + 1] += pre[j];
    }
    __syncthreads();
}

template <typename R, int NC, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 4) k_spread_rt_multi(const se_tile_args* __restrict__ av,
                                                                    const int* __restrict__ boff, int n)
{
    __shared__ se_rt_lds<R, NC, false> s;
    const int g = se_xcd_block(blockIdx.x, gridDim.x);
    const int j = job_of(boff, n, g);
    spread_rt_tile<R, NC, TG, false>(av[j], s, g - boff[j], 0, av[j].chunk);
}

template <typename R, int NC, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 4) k_spread_rt_extra_multi(const se_tile_args* __restrict__ av, int n)
{
    __shared__ se_rt_lds<R, NC, false> s;
    __shared__ int pre[SE_MULTI_MAX + 1];
    extra_prefix(av, n, pre);
    const int items = pre[n];
    for (int e = blockIdx.x; e < items; e += gridDim.x) {
        const int j = job_of(pre, n, e);
        const se_tile_args& a = av[j];
        const int ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
        const int le = e - pre[j];
        const int tile = rt_extra_tile(a.xoff, ntiles, le);
        const int c0 = (1 + le - a.xoff[tile]) * a.chunk;
        spread_rt_tile<R, NC, TG, true>(a, s, tile, c0, c0 + a.chunk);
        __syncthreads();
    }
}

template <typename R, int NCG, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 3) k_gather_rt_multi(const se_tile_args* __restrict__ av,
                                                                    const int* __restrict__ boff, int n)
{
    __shared__ se_rt_lds<R, NCG, true> s;
    const int g = se_xcd_block(blockIdx.x, gridDim.x);
    const int j = job_of(boff, n, g);
    gather_rt_tile<R, NCG, TG>(av[j], s, g - boff[j], 0, av[j].chunk);
}

template <typename R, int NCG, bool TG>
__global__ void __launch_bounds__(SE_RT_THREADS, 3) k_gather_rt_extra_multi(const se_tile_args* __restrict__ av, int n)
{
    __shared__ se_rt_lds<R, NCG, true> s;
    __shared__ int pre[SE_MULTI_MAX + 1];
    extra_prefix(av, n, pre);
    const int items = pre[n];
    for (int e = blockIdx.x; e < items; e += gridDim.x) {
        const int j = job_of(pre, n, e);
        const se_tile_args& a = av[j];
        const int ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
        const int le = e - pre[j];
        const int tile = rt_extra_tile(a.xoff, ntiles, le);
        const int c0 = (1 + le - a.xoff[tile]) * a.chunk;
        gather_rt_tile<R, NCG, TG>(a, s, tile, c0, c0 + a.chunk);
        __syncthreads();
    }
}

// Candidates of every tile (the same runs as rt_build_runs, one thread per
// tile) -> the number of items beyond the tile's first.
__global__ void k_rt_count(se_tile_args a, int ntiles, int* __restrict__ cnt)
{
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const se_grid_geom& g = a.g;
    int t0[3], te[3], b0[3], nbr[3];
    tile_origin_at(tile, a.ntile, SE_RT_TX, SE_RT_TY, SE_RT_TZ, g, t0, te);
    halo_bins(g, t0, te, a.P, b0, nbr);
    int kx0 = 0, kx1 = 0;
    if (g.periodic[0]) {
        kx0 = se_floordiv(b0[0], g.nb[0]);
        kx1 = se_floordiv(b0[0] + nbr[0] - 1, g.nb[0]);
    }
    const int nseg = nbr[0] > 0 ? kx1 - kx0 + 1 : 0;
    const int nslots = nbr[1] * nbr[2] * nseg;
    int total = 0;
    for (int slot = 0; slot < nslots; slot++) {
        const int row = slot / nseg, k = kx0 + slot % nseg;
        const int uy = b0[1] + row % nbr[1], uz = b0[2] + row / nbr[1];
        const int wy = g.periodic[1] ? uy - se_floordiv(uy, g.nb[1]) * g.nb[1] : uy;
        const int wz = g.periodic[2] ? uz - se_floordiv(uz, g.nb[2]) * g.nb[2] : uz;
        int lo = b0[0], hi = b0[0] + nbr[0] - 1;
        if (g.periodic[0]) {
            lo = max(lo, k * g.nb[0]);
            hi = min(hi, (k + 1) * g.nb[0] - 1);
        }
        const int wx0 = lo - k * g.nb[0];
        const int rowbase = (wz * g.nb[1] + wy) * g.nb[0];
        total += a.start[rowbase + wx0 + (hi - lo + 1)] - a.start[rowbase + wx0];
    }
    cnt[tile] = total > a.chunk ? (total - 1) / a.chunk : 0;
}

template <typename K>
void set_lds(K kern, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Candidates per work item of the register-tiled kernels: at least 16
// batches.  When the grid has tiles enough to fill the chip several times
// over, a tile is split only well above the mean candidate count of a
// uniform system (three times it), so that only tiles over dense clusters
// split; on grids with few tiles the 16-batch items also add parallelism.
constexpr int kRtChunk = 16 * SE_RT_KB;
constexpr unsigned kRtExtraBlocks = 1024;
constexpr int64_t kRtManyTiles = 8192;

int rt_chunk(const se_plan* p, int64_t npts)
{
    if (p->shape_tile_items > 0) return p->shape_tile_items * SE_RT_KB;
    const int64_t ntiles = (int64_t)p->ntile[0] * p->ntile[1] * p->ntile[2];
    if (ntiles < kRtManyTiles) return kRtChunk;
    const se_grid_geom& g = p->g;
    const int T[3] = {SE_RT_TX, SE_RT_TY, SE_RT_TZ};
    double frac = 1.0;  // halo bins of a tile / all bins, per axis
    for (int d = 0; d < 3; d++) {
        const int nbr = std::min((T[d] + p->par.P - 2) / g.B[d] + 2, g.nb[d]);
        frac *= (double)nbr / g.nb[d];
    }
    const double mean = frac * (double)npts;
    const int64_t c = ((int64_t)std::ceil(3.0 * mean / SE_RT_KB)) * SE_RT_KB;
    return (int)std::max<int64_t>(kRtChunk, std::min<int64_t>(c, 1 << 20));
}

se_tile_args make_args(const se_plan* p, bool gather, int slot)
{
    se_tile_args a;
    a.g = p->g;
    a.xs = gather && !p->tas ? p->d_tgt : p->d_src;
    a.n = gather ? p->nt : p->ns;
    a.start = gather && !p->tas ? p->d_tgt_start : p->d_src_start;
    a.pkb = p->d_pkb;
    a.P = p->par.P;
    a.nu = p->par.nu_deg;
    a.tg_c = p->par.window == SE_WINDOW_TG ? 4.0 * p->par.alpha / ((double)a.P * a.P) : 0.0;
    a.chunk = rt_chunk(p, a.n);
    a.xoff = gather && !p->tas ? p->d_rtx_t : p->d_rtx_s;
    for (int d = 0; d < 3; d++) a.ntile[d] = p->ntile[d];
    a.grid = se_slot_grid(p, slot);
    a.fs = se_slot_fs(p, slot);
    a.u = se_slot_uF(p, slot);
    return a;
}

template <typename R, int NC, int TX, int TY, int TZ>
void launch_spread(const se_plan* p, int slot, hipStream_t s)
{
    se_tile_args a = make_args(p, false, slot);
    size_t lds = SE_MAX_P * (SE_MAX_NU + 1) * sizeof(double) + (size_t)NC * TX * TY * TZ * sizeof(R);
    auto kern = k_spread<R, NC, TX, TY, TZ>;
    set_lds(kern, lds);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(SE_TILE_THREADS), lds, s, a);
}

template <typename R, int TX, int TY, int TZ>
void launch_gather(const se_plan* p, int slot, hipStream_t s)
{
    se_tile_args a = make_args(p, true, slot);
    size_t lds = SE_MAX_P * (SE_MAX_NU + 1) * sizeof(double) + (size_t)3 * TX * TY * TZ * sizeof(R);
    auto kern = k_gather<R, TX, TY, TZ>;
    set_lds(kern, lds);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(SE_TILE_THREADS), lds, s, a);
}

}  // namespace

// Tile shape used by both kernels (grid points per axis).
void se_tile_shape(int ncomp, bool fp32, int* tile)
{
    (void)ncomp;
    (void)fp32;
    tile[0] = SE_RT_TX;
    tile[1] = SE_RT_TY;
    tile[2] = SE_RT_TZ;
}

// The register-tiled kernels keep one slot per (halo bin row, x segment) in
// LDS; bound the count for this grid.
bool se_rt_fits(const se_plan* p)
{
    const se_grid_geom& g = p->g;
    const int T[3] = {SE_RT_TX, SE_RT_TY, SE_RT_TZ};
    int nbr[3];
    for (int d = 0; d < 3; d++) {
        nbr[d] = (T[d] + p->par.P - 2) / g.B[d] + 2;
        if (!g.periodic[d]) nbr[d] = std::min(nbr[d], g.nb[d]);
    }
    const int nseg = g.periodic[0] ? (nbr[0] + g.nb[0] - 1) / g.nb[0] + 1 : 1;
    return (int64_t)nbr[1] * nbr[2] * nseg <= SE_RT_MAXSLOTS && p->par.P <= SE_MAX_P;
}

template <typename R, int NC>
void launch_spread_rt(const se_plan* p, int slot, hipStream_t s)
{
    se_tile_args a = make_args(p, false, slot);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    if (a.tg_c > 0.0) {
        hipLaunchKernelGGL((k_spread_rt<R, NC, true>), dim3(nb), dim3(SE_RT_THREADS), 0, s, a);
        hipLaunchKernelGGL((k_spread_rt_extra<R, NC, true>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, a,
                           (int)nb);
    } else {
        hipLaunchKernelGGL((k_spread_rt<R, NC, false>), dim3(nb), dim3(SE_RT_THREADS), 0, s, a);
        hipLaunchKernelGGL((k_spread_rt_extra<R, NC, false>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, a,
                           (int)nb);
    }
}

template <typename R, int NCG>
void launch_gather_rt(const se_plan* p, int slot, hipStream_t s)
{
    se_tile_args a = make_args(p, true, slot);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    if (a.tg_c > 0.0) {
        hipLaunchKernelGGL((k_gather_rt<R, NCG, true>), dim3(nb), dim3(SE_RT_THREADS), 0, s, a);
        hipLaunchKernelGGL((k_gather_rt_extra<R, NCG, true>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, a,
                           (int)nb);
    } else {
        hipLaunchKernelGGL((k_gather_rt<R, NCG, false>), dim3(nb), dim3(SE_RT_THREADS), 0, s, a);
        hipLaunchKernelGGL((k_gather_rt_extra<R, NCG, false>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, a,
                           (int)nb);
    }
}

void se_launch_tile_prep(const se_plan* p, hipStream_t s)
{
    if (!se_rt_fits(p)) return;
    const int ntiles = p->ntile[0] * p->ntile[1] * p->ntile[2];
    for (int which = 0; which < (p->tas ? 1 : 2); which++) {
        se_tile_args a = make_args(p, which == 1, 0);
        int* cnt = which == 1 ? p->d_rtx_t : p->d_rtx_s;
        hipLaunchKernelGGL(k_rt_count, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, a, ntiles, cnt);
        se_launch_scan_excl(cnt, ntiles, s);
    }
}

// slot0 .. slot0 + nslot - 1: right-hand sides of the current chunk (two
// stokeslet/rotlet slots are gridded together as six components)
void se_launch_spread(const se_plan* p, int slot0, int nslot, hipStream_t s)
{
    if (se_rt_fits(p)) {
        if (p->ncomp == 3 && nslot == 2) {
            if (p->fp32) launch_spread_rt<float, 6>(p, slot0, s);
            else launch_spread_rt<double, 6>(p, slot0, s);
            return;
        }
        for (int k = 0; k < nslot; k++) {
            if (p->fp32) {
                if (p->ncomp == 3) launch_spread_rt<float, 3>(p, slot0 + k, s);
                else launch_spread_rt<float, 6>(p, slot0 + k, s);
            } else {
                if (p->ncomp == 3) launch_spread_rt<double, 3>(p, slot0 + k, s);
                else launch_spread_rt<double, 6>(p, slot0 + k, s);
            }
        }
        return;
    }
    for (int k = 0; k < nslot; k++) {
        if (p->fp32) {
            if (p->ncomp == 3) launch_spread<float, 3, 16, 16, 8>(p, slot0 + k, s);
            else launch_spread<float, 6, 16, 16, 8>(p, slot0 + k, s);
        } else {
            if (p->ncomp == 3) launch_spread<double, 3, 16, 16, 8>(p, slot0 + k, s);
            else launch_spread<double, 6, 16, 16, 8>(p, slot0 + k, s);
        }
    }
}

void se_launch_gather(const se_plan* p, int slot0, int nslot, hipStream_t s)
{
    if (se_rt_fits(p)) {
        if (nslot == 2) {
            if (p->fp32) launch_gather_rt<float, 6>(p, slot0, s);
            else launch_gather_rt<double, 6>(p, slot0, s);
            return;
        }
        for (int k = 0; k < nslot; k++) {
            if (p->fp32) launch_gather_rt<float, 3>(p, slot0 + k, s);
            else launch_gather_rt<double, 3>(p, slot0 + k, s);
        }
        return;
    }
    for (int k = 0; k < nslot; k++) {
        if (p->fp32) launch_gather<float, 16, 16, 8>(p, slot0 + k, s);
        else launch_gather<double, 16, 16, 8>(p, slot0 + k, s);
    }
}

// ---------------------------------------------------------------------------
// Jobs of merged batches.  Variant: bit 0 FP32 grid, bit 1 truncated
// Gaussian, bits 2.. the components per pass (3 or 6), as the single-plan
// launches above choose them.
namespace {

void add_tile_job(const se_plan* p, bool gather, int slot, int nc, std::vector<se_job>* out)
{
    se_job j;
    j.family = gather ? SE_JOB_GATHER : SE_JOB_SPREAD;
    const se_tile_args a = make_args(p, gather, slot);
    j.variant = (p->fp32 ? 1 : 0) | (a.tg_c > 0.0 ? 2 : 0) | (nc << 2);
    j.blocks = p->ntile[0] * p->ntile[1] * p->ntile[2];
    j.args.resize(sizeof(se_tile_args));
    std::memcpy(j.args.data(), &a, sizeof(a));
    out->push_back(std::move(j));
}

template <typename R, int NC, bool TG>
void tile_multi(bool gather, const void* args, const int* boff, int n, int blocks, hipStream_t s)
{
    const se_tile_args* av = (const se_tile_args*)args;
    if (gather) {
        hipLaunchKernelGGL((k_gather_rt_multi<R, NC, TG>), dim3(blocks), dim3(SE_RT_THREADS), 0, s, av, boff, n);
        hipLaunchKernelGGL((k_gather_rt_extra_multi<R, NC, TG>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, av,
                           n);
    } else {
        hipLaunchKernelGGL((k_spread_rt_multi<R, NC, TG>), dim3(blocks), dim3(SE_RT_THREADS), 0, s, av, boff, n);
        hipLaunchKernelGGL((k_spread_rt_extra_multi<R, NC, TG>), dim3(kRtExtraBlocks), dim3(SE_RT_THREADS), 0, s, av,
                           n);
    }
}

template <typename R, bool TG>
void tile_multi_nc(bool gather, int nc, const void* args, const int* boff, int n, int blocks, hipStream_t s)
{
    if (nc == 6) tile_multi<R, 6, TG>(gather, args, boff, n, blocks, s);
    else tile_multi<R, 3, TG>(gather, args, boff, n, blocks, s);
}

}  // namespace

bool se_tile_jobs(const se_plan* p, bool gather, int nslot, std::vector<se_job>* out)
{
    if (!se_rt_fits(p)) return false;
    if (gather) {
        if (nslot == 2) add_tile_job(p, true, 0, 6, out);
        else
            for (int k = 0; k < nslot; k++) add_tile_job(p, true, k, 3, out);
    } else {
        if (p->ncomp == 3 && nslot == 2) add_tile_job(p, false, 0, 6, out);
        else
            for (int k = 0; k < nslot; k++) add_tile_job(p, false, k, p->ncomp, out);
    }
    return true;
}

void se_tile_launch_multi(int family, int variant, const void* args, const int* boff, int n, int blocks,
                          hipStream_t s)
{
    if (n <= 0 || n > SE_MULTI_MAX) return;
    const bool gather = family == SE_JOB_GATHER;
    const bool fp32 = variant & 1, tg = variant & 2;
    const int nc = variant >> 2;
    if (fp32) {
        if (tg) tile_multi_nc<float, true>(gather, nc, args, boff, n, blocks, s);
        else tile_multi_nc<float, false>(gather, nc, args, boff, n, blocks, s);
    } else {
        if (tg) tile_multi_nc<double, true>(gather, nc, args, boff, n, blocks, s);
        else tile_multi_nc<double, false>(gather, nc, args, boff, n, blocks, s);
    }
}
