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
    int bid = blockIdx.x;
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

template <typename R, int NC, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_spread(se_tile_args a)
{
    extern __shared__ double smem_d[];
    constexpr int TV = TX * TY * TZ;
    double* s_pkb = smem_d;
    R* acc = (R*)(smem_d + SE_MAX_P * (SE_MAX_NU + 1));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin(a.ntile, TX, TY, TZ, g, t0, te);
    for (int i = tid; i < NC * TV; i += 256) acc[i] = (R)0;
    for (int i = tid; i < a.P * (a.nu + 1); i += 256) s_pkb[i] = a.pkb[i];
    __syncthreads();

    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int nrange = nbr[0] * nbr[1] * nbr[2];
    const R* fs = (const R*)a.fs;
    const int64_t n = a.n;
    for (int r = wave; r < nrange; r += 4) {
        int ub[3] = {b0[0] + r % nbr[0], b0[1] + (r / nbr[0]) % nbr[1], b0[2] + r / (nbr[0] * nbr[1])};
        int shift[3];
        int bin = wrap_bin(g, ub, shift);
        int s0 = a.start[bin], s1 = a.start[bin + 1];
        for (int s = s0; s < s1; s++) {
            double xp[3] = {a.xs[s], a.xs[n + s], a.xs[2 * n + s]};
            se_isect q;
            if (!point_isect(g, xp, shift, t0, te, a.P, q)) continue;
            R w = (R)0;
            if (lane < q.ex[0])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[0] + lane, (R)(1.0 - q.t[0]));
            else if (lane < q.ex[0] + q.ex[1])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[1] + lane - q.ex[0], (R)(1.0 - q.t[1]));
            else if (lane < q.ex[0] + q.ex[1] + q.ex[2])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[2] + lane - q.ex[0] - q.ex[1], (R)(1.0 - q.t[2]));
            R f[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) f[c] = fs[c * n + s];
            const int nxy = q.ex[0] * q.ex[1];
            const int zl = q.lo[2] - t0[2], yl = q.lo[1] - t0[1], xl = q.lo[0] - t0[0];
            for (int base = 0; base < nxy; base += 64) {
                int idx = base + lane;
                bool act = idx < nxy;
                int idc = act ? idx : 0;
                int iy = idc / q.ex[0];
                int ix = idc - iy * q.ex[0];
                R wx = shfl_r(w, ix);
                R wy = shfl_r(w, q.ex[0] + iy);
                R gv[NC];
#pragma unroll
                for (int c = 0; c < NC; c++) gv[c] = wx * wy * f[c];
                int lb = (zl * TY + yl + iy) * TX + xl + ix;
                for (int iz = 0; iz < q.ex[2]; iz++) {
                    R wz = se_readlane(w, q.ex[0] + q.ex[1] + iz);
                    if (act) {
#pragma unroll
                        for (int c = 0; c < NC; c++) atomicAdd(&acc[c * TV + lb + iz * TX * TY], wz * gv[c]);
                    }
                }
            }
        }
    }
    __syncthreads();
    R* grid = (R*)a.grid;
    const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
    const int64_t vol = plane * g.Mg[2];
    for (int i = tid; i < TV; i += 256) {
        int ix = i % TX, iy = (i / TX) % TY, iz = i / (TX * TY);
        if (ix < te[0] && iy < te[1] && iz < te[2]) {
            int64_t o = (int64_t)(t0[2] + iz) * plane + (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix;
#pragma unroll
            for (int c = 0; c < NC; c++) grid[c * vol + o] = acc[c * TV + i];
        }
    }
}

template <typename R, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_gather(se_tile_args a)
{
    extern __shared__ double smem_d[];
    constexpr int TV = TX * TY * TZ;
    double* s_pkb = smem_d;
    R* tile = (R*)(smem_d + SE_MAX_P * (SE_MAX_NU + 1));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const se_grid_geom& g = a.g;
    int t0[3], te[3];
    tile_origin(a.ntile, TX, TY, TZ, g, t0, te);
    const R* grid = (const R*)a.grid;
    const int64_t plane = (int64_t)g.Mg[0] * g.Mg[1];
    const int64_t vol = plane * g.Mg[2];
    for (int i = tid; i < TV; i += 256) {
        int ix = i % TX, iy = (i / TX) % TY, iz = i / (TX * TY);
        bool in = ix < te[0] && iy < te[1] && iz < te[2];
        int64_t o = (int64_t)(t0[2] + iz) * plane + (int64_t)(t0[1] + iy) * g.Mg[0] + t0[0] + ix;
#pragma unroll
        for (int c = 0; c < 3; c++) tile[c * TV + i] = in ? grid[c * vol + o] : (R)0;
    }
    for (int i = tid; i < a.P * (a.nu + 1); i += 256) s_pkb[i] = a.pkb[i];
    __syncthreads();

    int b0[3], nbr[3];
    halo_bins(g, t0, te, a.P, b0, nbr);
    const int nrange = nbr[0] * nbr[1] * nbr[2];
    const int64_t n = a.n;
    for (int r = wave; r < nrange; r += 4) {
        int ub[3] = {b0[0] + r % nbr[0], b0[1] + (r / nbr[0]) % nbr[1], b0[2] + r / (nbr[0] * nbr[1])};
        int shift[3];
        int bin = wrap_bin(g, ub, shift);
        int s0 = a.start[bin], s1 = a.start[bin + 1];
        for (int s = s0; s < s1; s++) {
            double xp[3] = {a.xs[s], a.xs[n + s], a.xs[2 * n + s]};
            se_isect q;
            if (!point_isect(g, xp, shift, t0, te, a.P, q)) continue;
            R w = (R)0;
            if (lane < q.ex[0])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[0] + lane, (R)(1.0 - q.t[0]));
            else if (lane < q.ex[0] + q.ex[1])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[1] + lane - q.ex[0], (R)(1.0 - q.t[1]));
            else if (lane < q.ex[0] + q.ex[1] + q.ex[2])
                w = se_pkb_eval<R>(s_pkb, a.nu, q.qoff[2] + lane - q.ex[0] - q.ex[1], (R)(1.0 - q.t[2]));
            const int nxy = q.ex[0] * q.ex[1];
            const int zl = q.lo[2] - t0[2], yl = q.lo[1] - t0[1], xl = q.lo[0] - t0[0];
            R acc0 = 0, acc1 = 0, acc2 = 0;
            for (int base = 0; base < nxy; base += 64) {
                int idx = base + lane;
                bool act = idx < nxy;
                int idc = act ? idx : 0;
                int iy = idc / q.ex[0];
                int ix = idc - iy * q.ex[0];
                R wx = shfl_r(w, ix);
                R wy = shfl_r(w, q.ex[0] + iy);
                R wxy = act ? wx * wy : (R)0;
                int lb = (zl * TY + yl + iy) * TX + xl + ix;
                for (int iz = 0; iz < q.ex[2]; iz++) {
                    R wz = se_readlane(w, q.ex[0] + q.ex[1] + iz) * wxy;
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
            if (lane == 0) {
                atomicAdd(&a.u[s], (double)acc0);
                atomicAdd(&a.u[n + s], (double)acc1);
                atomicAdd(&a.u[2 * n + s], (double)acc2);
            }
        }
    }
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
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), lds, s, a);
}

template <typename R, int TX, int TY, int TZ>
void launch_gather(const se_plan* p, hipStream_t s)
{
    se_tile_args a = make_args(p, true);
    size_t lds = SE_MAX_P * (SE_MAX_NU + 1) * sizeof(double) + (size_t)3 * TX * TY * TZ * sizeof(R);
    auto kern = k_gather<R, TX, TY, TZ>;
    set_lds(kern, lds);
    unsigned nb = (unsigned)(p->ntile[0] * p->ntile[1] * p->ntile[2]);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), lds, s, a);
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
