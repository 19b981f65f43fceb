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

__device__ __forceinline__ void tile_origin(const int* ntile, int TX, int TY, int TZ, const se_grid_geom& g,
                                            int* t0, int* te)
{
    int bid = se_xcd_block(blockIdx.x, gridDim.x);
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
            const R w = pkb_weight<R>(s_pkb, qq, (R)(1.0 - tt));
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
            const R w = pkb_weight<R>(s_pkb, qq, (R)(1.0 - tt));
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

template <typename K>
void set_lds(K kern, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

se_tile_args make_args(const se_plan* p, bool gather)
{
    se_tile_args a;
    a.g = p->g;
    a.xs = gather && !p->tas ? p->d_tgt : p->d_src;
    a.n = gather ? p->nt : p->ns;
    a.start = gather && !p->tas ? p->d_tgt_start : p->d_src_start;
    a.pkb = p->d_pkb;
    a.P = p->par.P;
    a.nu = p->par.nu_deg;
    for (int d = 0; d < 3; d++) a.ntile[d] = p->ntile[d];
    a.grid = p->d_grid;
    a.fs = p->d_fs;
    a.u = p->d_uF;
    return a;
}

template <typename R, int NC, int TX, int TY, int TZ>
void launch_spread(const se_plan* p, hipStream_t s)
{
    se_tile_args a = make_args(p, false);
    size_t lds = SE_MAX_P * (SE_MAX_NU + 1) * sizeof(double) + (size_t)NC * TX * TY * TZ * sizeof(R);
    auto kern = k_spread<R, NC, TX, TY, TZ>;
    set_lds(kern, lds);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(SE_TILE_THREADS), lds, s, a);
}

template <typename R, int TX, int TY, int TZ>
void launch_gather(const se_plan* p, hipStream_t s)
{
    se_tile_args a = make_args(p, true);
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
    tile[0] = 16;
    tile[1] = 16;
    tile[2] = (ncomp == 6 && !fp32) ? 4 : 8;
}

void se_launch_spread(const se_plan* p, hipStream_t s)
{
    if (p->fp32) {
        if (p->ncomp == 3) launch_spread<float, 3, 16, 16, 8>(p, s);
        else launch_spread<float, 6, 16, 16, 8>(p, s);
    } else {
        if (p->ncomp == 3) launch_spread<double, 3, 16, 16, 8>(p, s);
        else launch_spread<double, 6, 16, 16, 4>(p, s);
    }
}

void se_launch_gather(const se_plan* p, hipStream_t s)
{
    if (p->fp32) {
        launch_gather<float, 16, 16, 8>(p, s);
    } else {
        if (p->ncomp == 3) launch_gather<double, 16, 16, 8>(p, s);
        else launch_gather<double, 16, 16, 4>(p, s);
    }
}
