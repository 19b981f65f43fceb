// se_real.hip -- real-space part (eq. real-space-potential-Dp) on the cell
// list, strength staging, FP64 reductions and the epilogue that adds the
// self term (eq. 3p-stokeslet-self-term), the non-periodic stresslet term
// (eq. k0-stresslet-3p) and scatters back to the caller's order.
#include <algorithm>
#include <cstring>
#include <cmath>

#include "se_device.h"

namespace {

const double kSqrtPi = 1.7724538509055160272981675;

struct se_real_args {
    se_grid_geom g;
    const double4* xt; // sorted targets [nt] (x, y, z, 0)
    int64_t nt;
    const double4* xs; // sorted sources [ns]
    int64_t ns;
    const double4* f;  // sorted strengths [ns] (f, or q for T)
    const double4* nrm;// sorted normals [ns] (T)
    const double* rtab;// radial-function table
    const int* start;  // source cell starts
    const int* tstart; // target cell starts
    double xi, rc2;
    double rscale;     // SE_RTAB_N / (table range in x = xi r)
    int Ra[3];         // anchor reach ceil(rc/h)+1
    int tas;
    double* u;         // [3][nt]
    int* flags;
};

constexpr int kRn = SE_RTAB_DEG + 1;

__device__ __forceinline__ double horner_tab(const double* c, double sg)
{
    double acc = c[SE_RTAB_DEG];
#pragma unroll
    for (int k = SE_RTAB_DEG - 1; k >= 0; k--) acc = acc * sg + c[k];
    return acc;
}

// u_j += G^R_{jl(m)}(r; xi) . f, eqs. (stokeslet-real), (rotlet-real),
// (stresslet-real), written with x = xi r through G(x) = erfc(x) +
// (2x/sqrt(pi)) e^{-x^2} and E(x) = e^{-x^2} (tabulated, see se_radial_table):
//   S:     (G/r)(f + r (r.f)/r^2) - (4 xi/sqrt(pi)) E f
//   Omega: (G/r^3) (f x r)
//   H:     (erfc(x)/r) f, per component
//   T:     -2 r (r.q)(r.nu)/r^4 * (3G + (4x^3/sqrt(pi)) E)/r
//          + (4 xi^3/sqrt(pi)) E (q (r.nu) + nu (r.q) + r (q.nu))
struct se_radial {
    double inv, x, G, E;
};

__device__ __forceinline__ se_radial real_radial(const double* tab, double xi, double rscale, double r2)
{
    se_radial q;
    q.inv = rsqrt(r2);
    q.x = xi * r2 * q.inv;
    const double xs = q.x * rscale;
    const int iv = min((int)xs, SE_RTAB_N - 1);
    const double sg = 2.0 * (xs - iv) - 1.0;
    q.G = horner_tab(tab + iv * kRn, sg);
    q.E = horner_tab(tab + (SE_RTAB_N + iv) * kRn, sg);
    return q;
}

template <int KER>
__device__ __forceinline__ void real_apply(const se_radial& q, double xi, const double* r, const double* f,
                                           const double* nu, double* u)
{
    const double inv = q.inv;
    if constexpr (KER == SE_STOKESLET) {
        const double c1 = q.G * inv;
        const double c2 = (4.0 / kSqrtPi) * xi * q.E;
        const double rf = (r[0] * f[0] + r[1] * f[1] + r[2] * f[2]) * inv * inv;
#pragma unroll
        for (int j = 0; j < 3; j++) u[j] += c1 * (f[j] + r[j] * rf) - c2 * f[j];
    } else if constexpr (KER == SE_HARMONIC) {
        // erfc(x)/r = (G - (2x/sqrt(pi)) E)/r per component
        const double c1 = (q.G - (2.0 / kSqrtPi) * q.x * q.E) * inv;
#pragma unroll
        for (int j = 0; j < 3; j++) u[j] += c1 * f[j];
    } else if constexpr (KER == SE_ROTLET) {
        const double c1 = q.G * inv * inv * inv;
        u[0] += c1 * (f[1] * r[2] - f[2] * r[1]);
        u[1] += c1 * (f[2] * r[0] - f[0] * r[2]);
        u[2] += c1 * (f[0] * r[1] - f[1] * r[0]);
    } else {
        const double x = q.x;
        const double c1 = (3.0 * q.G + (4.0 / kSqrtPi) * x * x * x * q.E) * inv;
        const double c2 = (4.0 / kSqrtPi) * xi * xi * xi * q.E;
        const double rq = r[0] * f[0] + r[1] * f[1] + r[2] * f[2];
        const double rv = r[0] * nu[0] + r[1] * nu[1] + r[2] * nu[2];
        const double qv = f[0] * nu[0] + f[1] * nu[1] + f[2] * nu[2];
        const double i2 = inv * inv;
        const double a = -2.0 * rq * rv * i2 * i2 * c1;
#pragma unroll
        for (int j = 0; j < 3; j++) u[j] += a * r[j] + c2 * (f[j] * rv + nu[j] * rq + r[j] * qv);
    }
}

// u_j += G^R_{jl(m)}(r; xi) . f, eqs. (stokeslet-real), (rotlet-real),
// (stresslet-real), written with x = xi r through G(x) = erfc(x) +
// (2x/sqrt(pi)) e^{-x^2} and E(x) = e^{-x^2} (tabulated, see se_radial_table):
//   S:     (G/r)(f + r (r.f)/r^2) - (4 xi/sqrt(pi)) E f
//   Omega: (G/r^3) (f x r)
//   T:     -2 r (r.q)(r.nu)/r^4 * (3G + (4x^3/sqrt(pi)) E)/r
//          + (4 xi^3/sqrt(pi)) E (q (r.nu) + nu (r.q) + r (q.nu))
template <int KER>
__device__ __forceinline__ void real_pair(const double* tab, double xi, double rscale, const double* r, double r2,
                                          const double* f, const double* nu, double* u)
{
    real_apply<KER>(real_radial(tab, xi, rscale, r2), xi, r, f, nu, u);
}

// Persistent workgroups of 4 wavefronts; each wavefront walks a contiguous
// range of target cells (XCD-aware), taking up to 64 targets of a cell at a
// time.  The cell's neighbour bins form rows (by, bz) of consecutive x bins;
// each row, per x run with one image shift, is a contiguous range of the
// sorted sources.  Lanes take one row each and scan their ranges in lock
// step: every candidate source is loaded once and tested against all targets
// of the cell, so the neighbourhood is read once per cell, not once per
// target.  Hits |r| < rc are compacted with a ballot into a per-wave LDS queue
// of (target, source, image shift); every 64 queued pairs are evaluated by
// the 64 lanes together (full SIMD width) and added to per-target LDS
// accumulators.
#define SE_RQ 128
#define SE_REAL_BLOCKS 2048
#define SE_RT 64

__device__ __forceinline__ int pack_shift(int kx, int ky, int kz)
{
    return (kx + 64) | ((ky + 64) << 7) | ((kz + 64) << 14);
}

struct se_real_lds {
    int qs[SE_RQ];        // queued source index
    int qk[SE_RQ];        // queued (target << 21) | packed image shift
    double4 tp[SE_RT];    // target positions of the current chunk
    double acc[3][SE_RT]; // per-target accumulators
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KER>
__device__ __forceinline__ void eval_queue(const se_real_args& a, const double* tab, se_real_lds& L, int cnt,
                                           int lane)
{
    wave_sync();
    if (lane < cnt) {
        const se_grid_geom& g = a.g;
        const int s = L.qs[lane];
        const int pk = L.qk[lane];
        const int j = pk >> 21;
        const int kx = (pk & 127) - 64, ky = ((pk >> 7) & 127) - 64, kz = ((pk >> 14) & 127) - 64;
        const double4 p = a.xs[s];
        const double4 tq = L.tp[j];
        double r[3] = {tq.x - (p.x + kx * g.L[0]), tq.y - (p.y + ky * g.L[1]), tq.z - (p.z + kz * g.L[2])};
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double4 fv = a.f[s];
        double f[3] = {fv.x, fv.y, fv.z};
        double nu[3] = {0.0, 0.0, 0.0};
        if (KER == SE_STRESSLET) {
            const double4 nv = a.nrm[s];
            nu[0] = nv.x;
            nu[1] = nv.y;
            nu[2] = nv.z;
        }
        double u[3] = {0.0, 0.0, 0.0};
        real_pair<KER>(tab, a.xi, a.rscale, r, r2, f, nu, u);
        atomicAdd(&L.acc[0][j], u[0]);
        atomicAdd(&L.acc[1][j], u[1]);
        atomicAdd(&L.acc[2][j], u[2]);
    }
}

// Targets [tb, tb + ntc) of one cell with bin coordinates cb.  Rows are
// trimmed to the sources that can lie within rc of the cell's box: a row
// (by, bz) is skipped when its y/z distance to the box reaches rc, otherwise
// its x range is cut to the remaining reach sqrt(rc^2 - dy^2 - dz^2).
template <int KER>
__device__ __forceinline__ void real_cell(const se_real_args& a, const double* tab, se_real_lds& L, int cb[3],
                                          int64_t tb, int ntc, int lane)
{
    const se_grid_geom& g = a.g;
    int a0[3], a1[3], blo[3], bhi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        a0[d] = cb[d] * g.B[d];
        a1[d] = min(a0[d] + g.B[d] - 1, g.Mg[d] - 1);
        blo[d] = se_floordiv(a0[d] - a.Ra[d], g.B[d]);
        bhi[d] = se_floordiv(a1[d] + a.Ra[d], g.B[d]);
        if (!g.periodic[d]) {
            blo[d] = max(blo[d], 0);
            bhi[d] = min(bhi[d], g.nb[d] - 1);
        }
    }
    if (lane < ntc) {
        L.tp[lane] = a.xt[tb + lane];
        L.acc[0][lane] = 0.0;
        L.acc[1][lane] = 0.0;
        L.acc[2][lane] = 0.0;
    }
    wave_sync();
    const int ny = max(bhi[1] - blo[1] + 1, 0), nz = max(bhi[2] - blo[2] + 1, 0);
    const int nrows = ny * nz;
    const double rc2 = a.rc2;
    // cell box (grid index space, unwrapped): [a0, a1 + 1) per axis
    int qn = 0;
    int coinc = 0;
    for (int rb = 0; rb < nrows; rb += 64) {
        const int row = rb + lane;
        int ky = 0, kz = 0, rowbase = 0, uxl = 1, uxh = 0;
        if (row < nrows) {
            const int by = blo[1] + row % ny, bz = blo[2] + row / ny;
            ky = g.periodic[1] ? se_floordiv(by, g.nb[1]) : 0;
            kz = g.periodic[2] ? se_floordiv(bz, g.nb[2]) : 0;
            const int wy = by - ky * g.nb[1], wz = bz - kz * g.nb[2];
            rowbase = (wz * g.nb[1] + wy) * g.nb[0];
            // distances (grid units) between the row's bins and the cell box in y and z
            const int y0 = by * g.B[1], y1 = y0 + g.B[1];
            const int z0 = bz * g.B[2], z1 = z0 + g.B[2];
            const double dy = max(0, max(y0 - (a1[1] + 1), a0[1] - y1)) * g.h[1];
            const double dz = max(0, max(z0 - (a1[2] + 1), a0[2] - z1)) * g.h[2];
            const double rem2 = rc2 - dy * dy - dz * dz;
            if (rem2 > 0.0) {
                const int rx = (int)ceil(sqrt(rem2) * g.invh[0]) + 1;
                uxl = se_floordiv(a0[0] - rx, g.B[0]);
                uxh = se_floordiv(a1[0] + rx, g.B[0]);
                uxl = max(uxl, blo[0]);
                uxh = min(uxh, bhi[0]);
            }
        }
        const double sy = ky * g.L[1], sz = kz * g.L[2];
        int ux = uxl;
        int s = 0, e = 0, pk = 0;
        double sx = 0.0;
        bool zero_row = false;
        while (true) {
            // refill exhausted lanes with their next run of consecutive bins
            while (s == e && ux <= uxh) {
                const int kx = g.periodic[0] ? se_floordiv(ux, g.nb[0]) : 0;
                const int wx0 = ux - kx * g.nb[0];
                const int run = min(uxh - ux + 1, g.nb[0] - wx0);
                s = a.start[rowbase + wx0];
                e = a.start[rowbase + wx0 + run];
                sx = kx * g.L[0];
                pk = pack_shift(kx, ky, kz);
                zero_row = kx == 0 && ky == 0 && kz == 0;
                ux += run;
            }
            const bool active = s < e;
            if (!__ballot(active)) break;
            const int sc = active ? s : 0;
            const double4 p = a.xs[sc];
            const double px = p.x + sx, py = p.y + sy, pz = p.z + sz;
            for (int j = 0; j < ntc; j++) {
                const double4 tq = L.tp[j];
                const double d0 = tq.x - px, d1 = tq.y - py, d2 = tq.z - pz;
                const double rr = d0 * d0 + d1 * d1 + d2 * d2;
                bool hit = active && rr < rc2;
                if (hit && rr == 0.0) {
                    // the excluded self term (targets are sources) or a coincident pair
                    if (!(a.tas && zero_row && (int64_t)sc == tb + j)) coinc = 1;
                    hit = false;
                }
                const uint64_t m = __ballot(hit);
                if (m) {
                    if (hit) {
                        const int rank = __popcll(m & ((1ull << lane) - 1ull));
                        L.qs[qn + rank] = sc;
                        L.qk[qn + rank] = pk | (j << 21);
                    }
                    qn += __popcll(m);
                    if (qn >= 64) {
                        eval_queue<KER>(a, tab, L, 64, lane);
                        const int rem = qn - 64;
                        int ts = 0, tk = 0;
                        if (lane < rem) {
                            ts = L.qs[64 + lane];
                            tk = L.qk[64 + lane];
                        }
                        wave_sync();
                        if (lane < rem) {
                            L.qs[lane] = ts;
                            L.qk[lane] = tk;
                        }
                        qn = rem;
                    }
                }
            }
            s += active ? 1 : 0;
        }
    }
    eval_queue<KER>(a, tab, L, qn, lane);
    wave_sync();
    if (__ballot(coinc) && lane == 0) atomicOr(a.flags, SE_FLAG_COINCIDENT);
    if (lane < ntc) {
        a.u[tb + lane] = L.acc[0][lane];
        a.u[a.nt + tb + lane] = L.acc[1][lane];
        a.u[2 * a.nt + tb + lane] = L.acc[2][lane];
    }
    wave_sync();
}

template <int KER>
__global__ void __launch_bounds__(256) k_real(se_real_args a)
{
    __shared__ double tab[2 * SE_RTAB_N * kRn];
    __shared__ se_real_lds lds[4];
    for (int i = threadIdx.x; i < 2 * SE_RTAB_N * kRn; i += 256) tab[i] = a.rtab[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const se_grid_geom& g = a.g;
    const int64_t nbins = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t w = (int64_t)se_xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
    const int64_t chunk = (nbins + nw - 1) / nw;
    const int64_t c0 = w * chunk, c1 = min(nbins, c0 + chunk);
    for (int64_t c = c0; c < c1; c++) {
        const int tb = a.tstart[c], te = a.tstart[c + 1];
        if (tb == te) continue;
        int cb[3] = {(int)(c % g.nb[0]), (int)((c / g.nb[0]) % g.nb[1]), (int)(c / ((int64_t)g.nb[0] * g.nb[1]))};
        for (int t0 = tb; t0 < te; t0 += SE_RT) real_cell<KER>(a, tab, lds[wave], cb, t0, min(SE_RT, te - t0), lane);
    }
}

// ---------------------------------------------------------------------------
// Blocked real-space sum.  One wavefront per block of TB^3 target bins (about
// 48 targets, one per lane).  The sources that can lie within rc of the
// block's box form runs of the sorted order (rows of bins trimmed to the
// remaining reach, split at periodic wraps); they are streamed through LDS 64
// at a time, the next batch's loads in flight while the current one is used.
// Each lane tests its target against the 64 staged sources (one broadcast
// read each) and keeps a 64-bit hit mask, then walks its own mask evaluating
// the pairs; the sums stay in registers, so there are no atomics and every
// candidate is read from HBM/L2 once per block.
#define SE_R2_SLOTS 320
#define SE_R2_TROWS 16

#define SE_R2_QCAP 512

template <int KER, int RB>
struct se_real2_lds {
    double cx[64], cy[64], cz[64];  // shifted candidate positions
    double fx[RB][64], fy[RB][64], fz[RB][64];  // strengths of the RB right-hand sides
    double nx[KER == SE_STRESSLET ? 64 : 1], ny[KER == SE_STRESSLET ? 64 : 1],
        nz[KER == SE_STRESSLET ? 64 : 1];  // normals (stresslet)
    double tx[64], ty[64], tz[64];  // target positions of the chunk
    double acc[3 * RB][64];
    unsigned short q[SE_R2_QCAP];   // queued pairs: (target lane << 6) | candidate slot
    int cid[64];      // sorted index when unshifted, else -1
    int run_beg[SE_R2_SLOTS];
    int run_pre[SE_R2_SLOTS + 1];
    int trow_beg[SE_R2_TROWS];
    int trow_pre[SE_R2_TROWS + 1];
};

struct se_real2_geom {
    int TB;          // target bins per block and axis
    int nbk[3];      // blocks per axis
    int64_t nblk;
    const int* work; // exclusive scan of the blocks' 64-target chunks (nblk + 1 entries)
};

// Block ib of TB^3 target bins: its bin range per axis.
__device__ __forceinline__ void real2_block(const se_grid_geom& g, const se_real2_geom& bg, int64_t blk, int* b0,
                                            int* b1)
{
    const int ib[3] = {(int)(blk % bg.nbk[0]), (int)((blk / bg.nbk[0]) % bg.nbk[1]),
                       (int)(blk / ((int64_t)bg.nbk[0] * bg.nbk[1]))};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        b0[d] = ib[d] * bg.TB;
        b1[d] = min(b0[d] + bg.TB, g.nb[d]) - 1;
    }
}

// Work items of the blocked sum are (block, chunk of 64 targets), so that a
// block holding a dense cluster is spread over many wavefronts: first the
// chunk count of every block ...
__global__ void k_real2_chunks(se_real_args a, se_real2_geom bg, int* __restrict__ cnt)
{
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= bg.nblk) return;
    const se_grid_geom& g = a.g;
    int b0[3], b1[3];
    real2_block(g, bg, blk, b0, b1);
    const int tnx = b1[0] - b0[0] + 1;
    int nt = 0;
    for (int bz = b0[2]; bz <= b1[2]; bz++)
        for (int by = b0[1]; by <= b1[1]; by++) {
            const int rowbase = (bz * g.nb[1] + by) * g.nb[0];
            nt += a.tstart[rowbase + b0[0] + tnx] - a.tstart[rowbase + b0[0]];
        }
    cnt[blk] = (nt + 63) / 64;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// ... then their exclusive scan in place (one workgroup, tiles of 4096
// counts: four per thread, a wavefront scan, the wavefront totals through
// LDS, and a carry across tiles); v[n] receives the total.
__global__ void __launch_bounds__(1024) k_scan_excl(int* __restrict__ v, int64_t n)
{
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int carry = 0;
    for (int64_t base = 0; base < n; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)t;
        int x[4];
#pragma unroll
        for (int k = 0; k < 4; k++) x[k] = i0 + k < n ? v[i0 + k] : 0;
        const int s4 = x[0] + x[1] + x[2] + x[3];
        const int incl = wave_incl_scan(s4, lane);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int wpre = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const int ws = wsum[k];
            wpre += k < wv ? ws : 0;
            tot += ws;
        }
        int run = carry + wpre + incl - s4;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (i0 + k < n) v[i0 + k] = run;
            run += x[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (t == 0) v[n] = carry;
}

template <int KER, int RB>
__device__ __forceinline__ void eval_queue2(const se_real_args& a, const double* tab, se_real2_lds<KER, RB>& L,
                                            int qn, int lane)
{
    wave_sync();
    for (int e0 = 0; e0 < qn; e0 += 64) {
        const int e = e0 + lane;
        if (e < qn) {
            const int qv = L.q[e];
            const int tl = qv >> 6, c = qv & 63;
            const double r[3] = {L.tx[tl] - L.cx[c], L.ty[tl] - L.cy[c], L.tz[tl] - L.cz[c]};
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const se_radial q = real_radial(tab, a.xi, a.rscale, r2);
            double nu[3] = {0.0, 0.0, 0.0};
            if constexpr (KER == SE_STRESSLET) {
                nu[0] = L.nx[c];
                nu[1] = L.ny[c];
                nu[2] = L.nz[c];
            }
#pragma unroll
            for (int k = 0; k < RB; k++) {
                const double f[3] = {L.fx[k][c], L.fy[k][c], L.fz[k][c]};
                double u[3] = {0.0, 0.0, 0.0};
                real_apply<KER>(q, a.xi, r, f, nu, u);
                atomicAdd(&L.acc[3 * k + 0][tl], u[0]);
                atomicAdd(&L.acc[3 * k + 1][tl], u[1]);
                atomicAdd(&L.acc[3 * k + 2][tl], u[2]);
            }
        }
    }
    wave_sync();
}

// One work item of the blocked sum: targets 64 chunk .. 64 chunk + 63 of
// block blk against every source within rc of the block.
template <int KER, int RB>
__device__ __forceinline__ void real2_item(const se_real_args& a, const se_real2_geom& bg, const double* tab,
                                           se_real2_lds<KER, RB>& L, int lane, int64_t blk, int chunk, int& coinc)
{
    const se_grid_geom& g = a.g;
    int b0[3], b1[3], a0[3], a1[3], blo[3], bhi[3];
    real2_block(g, bg, blk, b0, b1);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        a0[d] = b0[d] * g.B[d];
        a1[d] = min((b1[d] + 1) * g.B[d], g.Mg[d]) - 1;
        blo[d] = se_floordiv(a0[d] - a.Ra[d], g.B[d]);
        bhi[d] = se_floordiv(a1[d] + a.Ra[d], g.B[d]);
        if (!g.periodic[d]) {
            blo[d] = max(blo[d], 0);
            bhi[d] = min(bhi[d], g.nb[d] - 1);
        }
    }
    // ---- candidate runs
    const int ny = bhi[1] - blo[1] + 1, nz = bhi[2] - blo[2] + 1;
    int kx0 = 0, kx1 = 0;
    if (g.periodic[0]) {
        kx0 = se_floordiv(blo[0], g.nb[0]);
        kx1 = se_floordiv(bhi[0], g.nb[0]);
    }
    const int nseg = kx1 - kx0 + 1;
    const int nslots = ny * nz * nseg;
    const double rc2 = a.rc2;
    for (int slot = lane; slot < nslots; slot += 64) {
        const int row = slot / nseg, k = kx0 + slot % nseg;
        const int by = blo[1] + row % ny, bz = blo[2] + row / ny;
        const int ky = g.periodic[1] ? se_floordiv(by, g.nb[1]) : 0;
        const int kz = g.periodic[2] ? se_floordiv(bz, g.nb[2]) : 0;
        const int wy = by - ky * g.nb[1], wz = bz - kz * g.nb[2];
        const int y0 = by * g.B[1], y1 = y0 + g.B[1];
        const int z0 = bz * g.B[2], z1 = z0 + g.B[2];
        const double dy = max(0, max(y0 - (a1[1] + 1), a0[1] - y1)) * g.h[1];
        const double dz = max(0, max(z0 - (a1[2] + 1), a0[2] - z1)) * g.h[2];
        const double rem2 = rc2 - dy * dy - dz * dz;
        int len = 0, beg = 0;
        if (rem2 > 0.0) {
            const int rx = (int)ceil(sqrt(rem2) * g.invh[0]) + 1;
            int lo = max(se_floordiv(a0[0] - rx, g.B[0]), blo[0]);
            int hi = min(se_floordiv(a1[0] + rx, g.B[0]), bhi[0]);
            if (g.periodic[0]) {
                lo = max(lo, k * g.nb[0]);
                hi = min(hi, (k + 1) * g.nb[0] - 1);
            }
            if (lo <= hi) {
                const int rowbase = (wz * g.nb[1] + wy) * g.nb[0];
                const int wx0 = lo - k * g.nb[0];
                beg = a.start[rowbase + wx0];
                len = a.start[rowbase + wx0 + (hi - lo + 1)] - beg;
            }
        }
        L.run_beg[slot] = beg;
        L.run_pre[slot + 1] = len;
    }
    wave_sync();
    {
        const int per = (nslots + 63) / 64;
        const int c0 = lane * per, c1 = min(c0 + per, nslots);
        int sum = 0;
        for (int i = c0; i < c1; i++) sum += L.run_pre[i + 1];
        int run = wave_incl_scan(sum, lane) - sum;
        for (int i = c0; i < c1; i++) {
            run += L.run_pre[i + 1];
            L.run_pre[i + 1] = run;
        }
        if (lane == 0) L.run_pre[0] = 0;
    }
    // ---- target rows of the block
    const int tnx = b1[0] - b0[0] + 1, tny = b1[1] - b0[1] + 1, tnz = b1[2] - b0[2] + 1;
    const int ntrows = tny * tnz;
    {
        int cnt = 0;
        if (lane < ntrows) {
            const int by = b0[1] + lane % tny, bz = b0[2] + lane / tny;
            const int rowbase = (bz * g.nb[1] + by) * g.nb[0];
            const int tb = a.tstart[rowbase + b0[0]];
            L.trow_beg[lane] = tb;
            cnt = a.tstart[rowbase + b0[0] + tnx] - tb;
        }
        const int incl = wave_incl_scan(cnt, lane);
        if (lane < ntrows) L.trow_pre[lane + 1] = incl;
        if (lane == 0) L.trow_pre[0] = 0;
    }
    wave_sync();
    const int total = L.run_pre[nslots];
    const int ntarg = L.trow_pre[ntrows];
    for (int tc = 64 * chunk; tc < min(ntarg, 64 * chunk + 64); tc += 64) {
        const int ft = tc + lane;
        const bool tvalid = ft < ntarg;
        int tidx = 0;
        if (tvalid) {
            int r = 0;
            while (r + 1 < ntrows && L.trow_pre[r + 1] <= ft) r++;
            tidx = L.trow_beg[r] + (ft - L.trow_pre[r]);
        }
        const double4 tq = a.xt[tvalid ? tidx : 0];
        L.tx[lane] = tq.x;
        L.ty[lane] = tq.y;
        L.tz[lane] = tq.z;
#pragma unroll
        for (int k = 0; k < 3 * RB; k++) L.acc[k][lane] = 0.0;
        // prefetch registers for one candidate per lane
        double4 np = make_double4(0, 0, 0, 0), nn = np;
        double4 nf[RB];
#pragma unroll
        for (int k = 0; k < RB; k++) nf[k] = np;
        int nid = -1;
        auto load = [&](int cbase) {
            const int f = cbase + lane;
            if (f < total) {
                int lo = 0, hi = nslots;
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (L.run_pre[mid] <= f) lo = mid;
                    else hi = mid;
                }
                const int sidx = L.run_beg[lo] + (f - L.run_pre[lo]);
                // image shift of the slot (row, x segment), as in the run table
                const int row = lo / nseg;
                const int kx = g.periodic[0] ? kx0 + lo % nseg : 0;
                const int ky = g.periodic[1] ? se_floordiv(blo[1] + row % ny, g.nb[1]) : 0;
                const int kz = g.periodic[2] ? se_floordiv(blo[2] + row / ny, g.nb[2]) : 0;
                const double4 p = a.xs[sidx];
                np = make_double4(p.x + kx * g.L[0], p.y + ky * g.L[1], p.z + kz * g.L[2], 0.0);
#pragma unroll
                for (int k = 0; k < RB; k++) nf[k] = a.f[(int64_t)k * a.ns + sidx];
                if (KER == SE_STRESSLET) nn = a.nrm[sidx];
                nid = (kx == 0 && ky == 0 && kz == 0) ? sidx : -1;
            }
        };
        load(0);
        for (int cb = 0; cb < total; cb += 64) {
            L.cx[lane] = np.x;
            L.cy[lane] = np.y;
            L.cz[lane] = np.z;
#pragma unroll
            for (int k = 0; k < RB; k++) {
                L.fx[k][lane] = nf[k].x;
                L.fy[k][lane] = nf[k].y;
                L.fz[k][lane] = nf[k].z;
            }
            if constexpr (KER == SE_STRESSLET) {
                L.nx[lane] = nn.x;
                L.ny[lane] = nn.y;
                L.nz[lane] = nn.z;
            }
            L.cid[lane] = nid;
            wave_sync();
            if (cb + 64 < total) load(cb + 64);
            const int n = min(64, total - cb);
            // tests in groups of 8 (reads first, then arithmetic); the mask is
            // built as two 32-bit words with compile-time bit positions
            uint32_t mw[2] = {0u, 0u};
            for (int c8 = 0; c8 < n; c8 += 8) {
                double qx[8], qy[8], qz[8];
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    qx[k] = L.cx[c8 + k];
                    qy[k] = L.cy[c8 + k];
                    qz[k] = L.cz[c8 + k];
                }
                uint32_t bits = 0u, zbits = 0u;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const double d0 = tq.x - qx[k], d1 = tq.y - qy[k], d2 = tq.z - qz[k];
                    const double rr = d0 * d0 + d1 * d1 + d2 * d2;
                    const bool inb = tvalid && (c8 + k < n);
                    bits |= (inb && rr < rc2 && rr != 0.0) ? (1u << k) : 0u;
                    zbits |= (inb && rr == 0.0) ? (1u << k) : 0u;
                }
                if (__ballot(zbits != 0u)) {
                    // the excluded self term (targets are sources) or a coincident pair
#pragma unroll
                    for (int k = 0; k < 8; k++)
                        if (((zbits >> k) & 1u) && !(a.tas && L.cid[c8 + k] == tidx)) coinc = 1;
                }
                mw[c8 >> 5] |= bits << (c8 & 31);
            }
            uint64_t mask = ((uint64_t)mw[1] << 32) | mw[0];
            // Queue the hits round-robin over the targets (the k-th hit of every
            // target, then the (k+1)-th, ...), so a window of 64 queued pairs
            // holds (nearly) distinct targets, and evaluate 64 pairs per step
            // at full width with one LDS accumulation per component.
            int qn = 0;
            while (__ballot(mask != 0)) {
                const bool has = mask != 0;
                const uint64_t b = __ballot(has);
                const int nb = __popcll(b);
                if (qn + nb > SE_R2_QCAP) {
                    eval_queue2<KER, RB>(a, tab, L, qn, lane);
                    qn = 0;
                }
                if (has) {
                    const int c = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    L.q[qn + __popcll(b & ((1ull << lane) - 1ull))] = (unsigned short)((lane << 6) | c);
                }
                qn += nb;
            }
            eval_queue2<KER, RB>(a, tab, L, qn, lane);
            wave_sync();
        }
        if (tvalid) {
#pragma unroll
            for (int k = 0; k < 3 * RB; k++) a.u[(int64_t)k * a.nt + tidx] = L.acc[k][lane];
        }
        wave_sync();
    }
}

// The work items, in the order of the scanned offsets, are cut into eight
// contiguous ranges, one per XCD (workgroups are dealt to the XCDs
// round-robin), so that neighbouring blocks share an L2; the workgroups of
// an XCD stride through its range.  The grid is sized on the host for an
// upper bound of the item count (blocks + targets / 64) and at least 8.
template <int KER, int RB>
__global__ void __launch_bounds__(256) k_real2(se_real_args a, se_real2_geom bg)
{
    // the radial table (5.6 KB) is read through the L1 cache rather than
    // staged in LDS: the four waves' staging then fits three blocks per CU
    const double* tab = a.rtab;
    __shared__ se_real2_lds<KER, RB> lds[4];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwg = gridDim.x, xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    const int nx = nwg / 8 + (xcd < nwg % 8 ? 1 : 0);
    const int64_t items = bg.work[bg.nblk];
    const int64_t lo = items * xcd / 8, hi = items * (xcd + 1) / 8;
    int coinc = 0;
    for (int64_t w = lo + (int64_t)idx * 4 + wave; w < hi; w += (int64_t)nx * 4) {
        // item w -> (block, chunk): the last block whose offset is <= w
        // (empty blocks share their offset with the next one)
        int64_t blk = 0, top = bg.nblk;
        while (top - blk > 1) {
            const int64_t mid = (blk + top) >> 1;
            if (bg.work[mid] <= w) blk = mid;
            else top = mid;
        }
        real2_item<KER, RB>(a, bg, tab, lds[wave], lane, blk, (int)(w - bg.work[blk]), coinc);
    }
    if (__ballot(coinc) && lane == 0) atomicOr(a.flags, SE_FLAG_COINCIDENT);
}

// Sorted strengths: FP64 copy [3][ns] of f (or q) for the real-space sum and
// self term, the gridded components in grid precision [ncomp][ns]
// (f, or the symmetric part of q nu^T: xx, yy, zz, xy, xz, yz), and q.nu.
template <typename R>
__global__ void k_strengths(const double* __restrict__ f, const int* __restrict__ perm, int64_t n,
                            const double* __restrict__ nrm, int ncomp, double* __restrict__ f64,
                            R* __restrict__ fs, double* __restrict__ qn, double4* __restrict__ f4, int* flags)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    double v[3];
    bool bad = false;
    for (int c = 0; c < 3; c++) {
        v[c] = f[3 * o + c];
        if (!isfinite(v[c])) bad = true;
    }
    if (bad) {
        atomicOr(flags, SE_FLAG_NONFINITE);
        v[0] = v[1] = v[2] = 0.0;
    }
    for (int c = 0; c < 3; c++) f64[c * n + s] = v[c];
    f4[s] = make_double4(v[0], v[1], v[2], 0.0);
    if (ncomp == 3) {
        for (int c = 0; c < 3; c++) fs[c * n + s] = (R)v[c];
    } else {
        double nu[3] = {nrm[s], nrm[n + s], nrm[2 * n + s]};
        fs[0 * n + s] = (R)(v[0] * nu[0]);
        fs[1 * n + s] = (R)(v[1] * nu[1]);
        fs[2 * n + s] = (R)(v[2] * nu[2]);
        fs[3 * n + s] = (R)(0.5 * (v[0] * nu[1] + v[1] * nu[0]));
        fs[4 * n + s] = (R)(0.5 * (v[0] * nu[2] + v[2] * nu[0]));
        fs[5 * n + s] = (R)(0.5 * (v[1] * nu[2] + v[2] * nu[1]));
        qn[s] = v[0] * nu[0] + v[1] * nu[1] + v[2] * nu[2];
    }
}

// Deterministic FP64 reductions over the sources, in two fixed-order stages:
// out[0] = sum q.nu, out[1..3] = sum x (q.nu) (stresslet zero-mode term,
// eq. k0-stresslet-3p), out[4..6] = sum f (gauge terms of the stokeslet).
// Stage 1: block b reduces the contiguous chunk b into part[c * SE_RED_BLOCKS + b];
// stage 2: one block reduces the partials.
__global__ void __launch_bounds__(512) k_reduce_sources(const double* __restrict__ qn, const double* __restrict__ f,
                                                        const double* __restrict__ xs, int64_t n, int have_qn,
                                                        double* part)
{
    __shared__ double sm[7][512];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t chunk = (n + SE_RED_BLOCKS - 1) / SE_RED_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 512) {
        double q = have_qn ? qn[i] : 0.0;
        a[0] += q;
        a[1] += xs[i] * q;
        a[2] += xs[n + i] * q;
        a[3] += xs[2 * n + i] * q;
        a[4] += f[i];
        a[5] += f[n + i];
        a[6] += f[2 * n + i];
    }
    for (int c = 0; c < 7; c++) sm[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int w = 256; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 7; c++) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 7) part[threadIdx.x * SE_RED_BLOCKS + blockIdx.x] = sm[threadIdx.x][0];
}

__global__ void __launch_bounds__(SE_RED_BLOCKS) k_reduce_final(const double* __restrict__ part, double* out)
{
    __shared__ double sm[7][SE_RED_BLOCKS];
    for (int c = 0; c < 7; c++) sm[c][threadIdx.x] = part[c * SE_RED_BLOCKS + threadIdx.x];
    __syncthreads();
    for (int w = SE_RED_BLOCKS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 7; c++) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 7) out[threadIdx.x] = sm[threadIdx.x][0];
}

struct se_fin_args {
    int64_t nt;
    const int* perm;      // target sorted -> original
    const double* uF;     // [3][nt]
    const double* uR;
    const double* f64;    // sorted source strengths (self term; targets are sources)
    const double* xt;     // sorted targets
    const double* red;    // stresslet sums
    double self_c;        // -4 xi/sqrt(pi) (stokeslet, targets are sources) or 0
    double k0_c;          // -8 pi/|B| (D = 3 stresslet) or 0
    double gauge[3];      // constant added per component times sum f (stokeslet gauges)
    double* u;            // [nt][3] caller order (or null)
    double* u_real;
    double* u_four;
};

// Merged real-space sums of many plans (batches of systems): job j is
// (args, block geometry) of one plan and slot; its items follow the
// device-side scan of its blocks, and all jobs' items are split over the
// XCDs as in k_real2.
struct se_real_job {
    se_real_args a;
    se_real2_geom bg;
};
constexpr int kRealJobMax = 256;

template <int KER, int RB>
__global__ void __launch_bounds__(256) k_real2_multi(const se_real_job* __restrict__ jv, int n)
{
    __shared__ se_real2_lds<KER, RB> lds[4];
    __shared__ int pre[kRealJobMax + 1];
    for (int j = threadIdx.x; j < n; j += blockDim.x) pre[j + 1] = jv[j].bg.work[jv[j].bg.nblk];
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int j = 0; j < n; j++) pre[j + 1] += pre[j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwg = gridDim.x, xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    const int nx = nwg / 8 + (xcd < nwg % 8 ? 1 : 0);
    const int64_t items = pre[n];
    const int64_t lo = items * xcd / 8, hi = items * (xcd + 1) / 8;
    for (int64_t w = lo + (int64_t)idx * 4 + wave; w < hi; w += (int64_t)nx * 4) {
        int j = 0, top = n;  // the last job whose offset is <= w
        while (top - j > 1) {
            const int mid = (j + top) >> 1;
            if (pre[mid] <= w) j = mid;
            else top = mid;
        }
        const se_real_args& a = jv[j].a;
        const se_real2_geom& bg = jv[j].bg;
        const int64_t lw = w - pre[j];
        int64_t blk = 0, tb = bg.nblk;
        while (tb - blk > 1) {
            const int64_t mid = (blk + tb) >> 1;
            if (bg.work[mid] <= lw) blk = mid;
            else tb = mid;
        }
        int coinc = 0;
        real2_item<KER, RB>(a, bg, a.rtab, lds[wave], lane, blk, (int)(lw - bg.work[blk]), coinc);
        if (__ballot(coinc) && lane == 0) atomicOr(a.flags, SE_FLAG_COINCIDENT);
    }
}

__global__ void k_finalize(se_fin_args a)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nt) return;
    int64_t o = a.perm[t];
    for (int j = 0; j < 3; j++) {
        double ur = a.uR[j * a.nt + t];
        double uf = a.uF[j * a.nt + t];
        if (a.self_c != 0.0) uf += a.self_c * a.f64[j * a.nt + t];
        if (a.k0_c != 0.0) uf += a.k0_c * (a.xt[j * a.nt + t] * a.red[0] - a.red[1 + j]);
        uf += a.gauge[j] * a.red[4 + j];
        if (a.u) a.u[3 * o + j] = ur + uf;
        if (a.u_real) a.u_real[3 * o + j] = ur;
        if (a.u_four) a.u_four[3 * o + j] = uf;
    }
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

namespace {

// ------------------------------------------------- direct real-space reference
// All pairs, one thread per target, sources through LDS in tiles of 256.
// D = 3: the minimum image within rc <= min L / 2 (at most one image of a
// pair is that close) with the exact real-space kernels, eqs.
// (stokeslet-real), (rotlet-real), (stresslet-real), erfc(xi r)/r for the
// harmonic; D = 0: the free-space kernels (the same forms at xi = 0).
// The pair m = n is skipped when targets are sources; coincident distinct
// pairs are skipped and flagged.
struct se_dref_r_args {
    int D;
    double L[3];
    double xi, rc2;
    int64_t ns, nt;
    const double* xs;
    const double* f;
    const double* nu;
    const double* xt;
    int tas;
    double* u;
    int* flags;
};

template <int KER>
__global__ void __launch_bounds__(256) k_dref_real(se_dref_r_args a)
{
    constexpr int NN = KER == SE_STRESSLET ? 256 : 1;
    __shared__ double sx[256][3], sf[256][3], sn[NN][3];
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x[3] = {0.0, 0.0, 0.0};
    if (m < a.nt)
        for (int d = 0; d < 3; d++) x[d] = a.xt[3 * m + d];
    double acc[3] = {0.0, 0.0, 0.0};
    int coinc = 0;
    for (int64_t base = 0; base < a.ns; base += 256) {
        const int64_t n = base + threadIdx.x;
        if (n < a.ns)
            for (int d = 0; d < 3; d++) {
                sx[threadIdx.x][d] = a.xs[3 * n + d];
                sf[threadIdx.x][d] = a.f[3 * n + d];
                if constexpr (KER == SE_STRESSLET) sn[threadIdx.x][d] = a.nu[3 * n + d];
            }
        __syncthreads();
        const int cnt = (int)min((int64_t)256, a.ns - base);
        if (m < a.nt) {
            for (int j = 0; j < cnt; j++) {
                if (a.tas && base + j == m) continue;
                double r[3];
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    r[d] = x[d] - sx[j][d];
                    if (d < a.D) r[d] -= a.L[d] * rint(r[d] / a.L[d]);
                }
                const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                if (a.D > 0 && r2 >= a.rc2) continue;
                if (r2 == 0.0) {
                    coinc = 1;
                    continue;
                }
                se_radial q;
                q.inv = 1.0 / sqrt(r2);
                q.x = a.xi * r2 * q.inv;
                q.E = exp(-q.x * q.x);
                q.G = erfc(q.x) + (2.0 / kSqrtPi) * q.x * q.E;
                const double* nn = nullptr;
                if constexpr (KER == SE_STRESSLET) nn = sn[j];
                real_apply<KER>(q, a.xi, r, sf[j], nn, acc);
            }
        }
        __syncthreads();
    }
    if (m < a.nt)
        for (int d = 0; d < 3; d++) a.u[3 * m + d] = acc[d];
    if (coinc) atomicOr(a.flags, SE_FLAG_COINCIDENT);
}

// Zero modes k^P = 0 of the Fourier part for D = 2 and D = 1, in the closed
// forms of Appendix A.2 (eqs. 2p-rotlet-Q0, 2p-stokeslet-Q0,
// 2p-stresslet-Q0 and the harmonic's Q^{H,2P,(0)}) and Appendix B.2 (eqs.
// 1p-rotlet-Q0, 1p-stokeslet-Q0 with its limit, 1p-stresslet-Q0, and
// Q^{H,1P,(0)} with l_H = 1), over all pairs including m = n.
// E1 by its power series (x <= 1) and its continued fraction evaluated
// with the modified Lentz method (x > 1).
__device__ double dref_e1(double x)
{
    const double euler = 0.57721566490153286061;
    if (x <= 1.0) {
        double term = 1.0, sum = 0.0;
        for (int k = 1; k < 80; k++) {
            term *= -x / k;
            sum += term / k;
            if (fabs(term) < 1e-18 * k * fabs(sum)) break;
        }
        return -euler - log(x) - sum;
    }
    double b = x + 1.0, c = 1e300, d = 1.0 / b, h = d;
    for (int i = 1; i < 300; i++) {
        const double an = -(double)i * i;
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        const double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return h * exp(-x);
}

template <int KER>
__device__ __forceinline__ void dref_zero_2p(double xi, double r3, const double* f, const double* nu, double* u)
{
    const double e = exp(-xi * xi * r3 * r3), ef = erf(xi * r3);
    if constexpr (KER == SE_HARMONIC) {
        const double c = -2.0 * M_PI * (r3 * ef + e / (kSqrtPi * xi));
        for (int j = 0; j < 3; j++) u[j] += c * f[j];
    } else if constexpr (KER == SE_STOKESLET) {
        const double c = -2.0 * M_PI * (2.0 * r3 * ef + e / (kSqrtPi * xi));
        u[0] += c * f[0];
        u[1] += c * f[1];
    } else if constexpr (KER == SE_ROTLET) {
        const double c = 2.0 * M_PI * ef;
        u[0] += c * f[1];
        u[1] -= c * f[0];
    } else {
        const double c = -4.0 * M_PI * (ef + xi * r3 * e / kSqrtPi);
        u[0] += c * (f[0] * nu[2] + f[2] * nu[0]);
        u[1] += c * (f[1] * nu[2] + f[2] * nu[1]);
        u[2] += c * (f[0] * nu[0] + f[1] * nu[1] + f[2] * nu[2]);
    }
}

template <int KER>
__device__ __forceinline__ void dref_zero_1p(double xi, double r2, double r3, const double* f, const double* nu,
                                             double* u)
{
    const double euler = 0.57721566490153286061;
    const double rho2 = r2 * r2 + r3 * r3, V = xi * xi * rho2;
    if (rho2 == 0.0) {
        if constexpr (KER == SE_HARMONIC) {
            const double c = euler + log(xi * xi);
            for (int j = 0; j < 3; j++) u[j] += c * f[j];
        } else if constexpr (KER == SE_STOKESLET) {
            const double c = euler + log(xi * xi) - 1.0;
            u[0] += 2.0 * c * f[0];
            u[1] += c * f[1];
            u[2] += c * f[2];
        }
        return;  // rotlet and stresslet: zero
    }
    const double rho = sqrt(rho2), t2 = r2 / rho, t3 = r3 / rho;
    const double p1 = -expm1(-V);
    if constexpr (KER == SE_HARMONIC) {
        const double c = -(dref_e1(V) + log(rho2));
        for (int j = 0; j < 3; j++) u[j] += c * f[j];
    } else if constexpr (KER == SE_ROTLET) {
        const double c = 2.0 * p1 / rho;
        u[0] += c * (t3 * f[1] - t2 * f[2]);
        u[1] -= c * t3 * f[0];
        u[2] += c * t2 * f[0];
    } else if constexpr (KER == SE_STOKESLET) {
        const double p0 = dref_e1(V) + log(rho2) + 1.0;
        u[0] -= 2.0 * (p0 + p1) * f[0];
        u[1] -= (p0 + 2.0 * t3 * t3 * p1) * f[1] - 2.0 * t2 * t3 * p1 * f[2];
        u[2] -= -2.0 * t2 * t3 * p1 * f[1] + (p0 + 2.0 * t2 * t2 * p1) * f[2];
    } else {
        double p2;
        if (V < 0.05) {  // 1 - (1 + V) e^{-V} = sum_{n>=2} (-1)^n (n-1) V^n / n!
            double pw = V * V, fact = 2.0;
            p2 = 0.0;
            for (int n = 2; n < 24; n++) {
                p2 += ((n & 1) ? -1.0 : 1.0) * (n - 1) * pw / fact;
                pw *= V;
                fact *= n + 1;
            }
        } else {
            p2 = p1 - V * exp(-V);
        }
        const double R = -4.0 / rho;
        const double q112 = R * t2 * (2.0 * p1 - p2), q113 = R * t3 * (2.0 * p1 - p2);
        const double q222 = R * t2 * (3.0 * p1 - (t2 * t2 + 3.0 * t3 * t3) * p2);
        const double q223 = R * t3 * (p1 - (t3 * t3 - t2 * t2) * p2);
        const double q233 = R * t2 * (p1 - (t2 * t2 - t3 * t3) * p2);
        const double q333 = R * t3 * (3.0 * p1 - (3.0 * t2 * t2 + t3 * t3) * p2);
        const double* q = f;
        u[0] += q112 * (q[0] * nu[1] + q[1] * nu[0]) + q113 * (q[0] * nu[2] + q[2] * nu[0]);
        u[1] += q112 * q[0] * nu[0] + q222 * q[1] * nu[1] + q223 * (q[1] * nu[2] + q[2] * nu[1]) + q233 * q[2] * nu[2];
        u[2] += q113 * q[0] * nu[0] + q223 * q[1] * nu[1] + q233 * (q[1] * nu[2] + q[2] * nu[1]) + q333 * q[2] * nu[2];
    }
}

template <int KER>
__global__ void __launch_bounds__(256) k_dref_zero(se_dref_r_args a, double inv_area)
{
    constexpr int NN = KER == SE_STRESSLET ? 256 : 1;
    __shared__ double sx[256][3], sf[256][3], sn[NN][3];
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x[3] = {0.0, 0.0, 0.0};
    if (m < a.nt)
        for (int d = 0; d < 3; d++) x[d] = a.xt[3 * m + d];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t base = 0; base < a.ns; base += 256) {
        const int64_t n = base + threadIdx.x;
        if (n < a.ns)
            for (int d = 0; d < 3; d++) {
                sx[threadIdx.x][d] = a.xs[3 * n + d];
                sf[threadIdx.x][d] = a.f[3 * n + d];
                if constexpr (KER == SE_STRESSLET) sn[threadIdx.x][d] = a.nu[3 * n + d];
            }
        __syncthreads();
        const int cnt = (int)min((int64_t)256, a.ns - base);
        if (m < a.nt) {
            for (int j = 0; j < cnt; j++) {
                const double* nn = nullptr;
                if constexpr (KER == SE_STRESSLET) nn = sn[j];
                if (a.D == 2) dref_zero_2p<KER>(a.xi, x[2] - sx[j][2], sf[j], nn, acc);
                else dref_zero_1p<KER>(a.xi, x[1] - sx[j][1], x[2] - sx[j][2], sf[j], nn, acc);
            }
        }
        __syncthreads();
    }
    if (m < a.nt)
        for (int d = 0; d < 3; d++) a.u[3 * m + d] += acc[d] * inv_area;
}

// Source sums for the terms outside the lattice sums: sum f (3), sum q.nu,
// sum x_n (q.nu) (3); one workgroup, fixed order (deterministic).
__global__ void __launch_bounds__(1024) k_dref_sums(int64_t ns, const double* xs, const double* f, const double* nu,
                                                    int stresslet, double* out)
{
    __shared__ double red[7][1024];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = threadIdx.x; n < ns; n += 1024) {
        for (int d = 0; d < 3; d++) v[d] += f[3 * n + d];
        if (stresslet) {
            const double qn = f[3 * n] * nu[3 * n] + f[3 * n + 1] * nu[3 * n + 1] + f[3 * n + 2] * nu[3 * n + 2];
            v[3] += qn;
            for (int d = 0; d < 3; d++) v[4 + d] += xs[3 * n + d] * qn;
        }
    }
    for (int c = 0; c < 7; c++) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int c = 0; c < 7; c++) red[c][threadIdx.x] += red[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 7) out[threadIdx.x] = red[threadIdx.x][0];
}

// u += self term (targets are sources), the D = 3 stresslet k = 0 term
// (eq. k0-stresslet-3p) and the harmonic's neutralising background.
__global__ void k_dref_terms(int64_t nt, const double* xt, const double* f, int tas, double self_c, double k0_c,
                             double bg_c, const double* sums, double* u)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nt) return;
    for (int j = 0; j < 3; j++) {
        double v = bg_c * sums[j];
        if (tas) v += self_c * f[3 * m + j];
        if (k0_c != 0.0) v += k0_c * (xt[3 * m + j] * sums[3] - sums[4 + j]);
        u[3 * m + j] += v;
    }
}

}  // namespace

void se_launch_dref_real(int kernel, int D, const double* L, double xi, double rc, int64_t ns, const double* xs,
                         const double* f, const double* nu, int64_t nt, const double* xt, int tas, double* u,
                         int* flags, hipStream_t s)
{
    se_dref_r_args a;
    a.D = D;
    for (int d = 0; d < 3; d++) a.L[d] = L[d];
    a.xi = D == 0 ? 0.0 : xi;
    a.rc2 = rc * rc;
    a.ns = ns;
    a.nt = nt;
    a.xs = xs;
    a.f = f;
    a.nu = nu;
    a.xt = xt;
    a.tas = tas;
    a.u = u;
    a.flags = flags;
    const dim3 g((unsigned)((nt + 255) / 256));
    if (kernel == SE_STOKESLET) hipLaunchKernelGGL(k_dref_real<SE_STOKESLET>, g, dim3(256), 0, s, a);
    else if (kernel == SE_ROTLET) hipLaunchKernelGGL(k_dref_real<SE_ROTLET>, g, dim3(256), 0, s, a);
    else if (kernel == SE_HARMONIC) hipLaunchKernelGGL(k_dref_real<SE_HARMONIC>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_dref_real<SE_STRESSLET>, g, dim3(256), 0, s, a);
}

void se_launch_dref_zero(int kernel, int D, const double* L, double xi, int64_t ns, const double* xs,
                         const double* f, const double* nu, int64_t nt, const double* xt, double* u, hipStream_t s)
{
    if (D != 1 && D != 2) return;
    se_dref_r_args a{};
    a.D = D;
    a.xi = xi;
    a.ns = ns;
    a.nt = nt;
    a.xs = xs;
    a.f = f;
    a.nu = nu;
    a.xt = xt;
    a.u = u;
    const double inv_area = D == 2 ? 1.0 / (L[0] * L[1]) : 1.0 / L[0];
    const dim3 g((unsigned)((nt + 255) / 256));
    if (kernel == SE_STOKESLET) hipLaunchKernelGGL(k_dref_zero<SE_STOKESLET>, g, dim3(256), 0, s, a, inv_area);
    else if (kernel == SE_ROTLET) hipLaunchKernelGGL(k_dref_zero<SE_ROTLET>, g, dim3(256), 0, s, a, inv_area);
    else if (kernel == SE_HARMONIC) hipLaunchKernelGGL(k_dref_zero<SE_HARMONIC>, g, dim3(256), 0, s, a, inv_area);
    else hipLaunchKernelGGL(k_dref_zero<SE_STRESSLET>, g, dim3(256), 0, s, a, inv_area);
}

void se_launch_dref_terms(int kernel, int D, const double* L, double xi, int64_t ns, const double* xs,
                          const double* f, const double* nu, int64_t nt, const double* xt, int tas, double* sums,
                          double* u, hipStream_t s)
{
    if (D == 0) return;
    const double V = L[0] * L[1] * L[2];
    const double self_c = kernel == SE_STOKESLET ? -4.0 * xi / kSqrtPi : (kernel == SE_HARMONIC ? -2.0 * xi / kSqrtPi : 0.0);
    const double k0_c = kernel == SE_STRESSLET && D == 3 ? -8.0 * M_PI / V : 0.0;
    const double bg_c = kernel == SE_HARMONIC && D == 3 ? -M_PI / (V * xi * xi) : 0.0;
    hipLaunchKernelGGL(k_dref_sums, dim3(1), dim3(1024), 0, s, ns, xs, f, nu, kernel == SE_STRESSLET ? 1 : 0, sums);
    hipLaunchKernelGGL(k_dref_terms, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, nt, tas ? xs : xt, f, tas,
                       self_c, k0_c, bg_c, sums, u);
}

void se_launch_strengths(const se_plan* p, const double* f, int slot, hipStream_t s)
{
    double* f64 = se_slot_fs64(p, slot);
    double4* f4 = (double4*)se_slot_str4(p, slot);
    if (p->fp32)
        hipLaunchKernelGGL(k_strengths<float>, dim3(grid1d(p->ns, 256)), dim3(256), 0, s, f, p->d_src_perm, p->ns,
                           p->d_nrm, p->ncomp, f64, (float*)se_slot_fs(p, slot), f64 + 3 * p->ns, f4, p->d_flags);
    else
        hipLaunchKernelGGL(k_strengths<double>, dim3(grid1d(p->ns, 256)), dim3(256), 0, s, f, p->d_src_perm, p->ns,
                           p->d_nrm, p->ncomp, f64, (double*)se_slot_fs(p, slot), f64 + 3 * p->ns, f4, p->d_flags);
}

void se_launch_reductions(const se_plan* p, int slot, hipStream_t s)
{
    double* red = se_slot_red(p, slot);
    double* part = red + SE_RED_OUT;
    const double* f64 = se_slot_fs64(p, slot);
    hipLaunchKernelGGL(k_reduce_sources, dim3(SE_RED_BLOCKS), dim3(512), 0, s, f64 + 3 * p->ns, f64, p->d_src, p->ns,
                       p->kernel == SE_STRESSLET ? 1 : 0, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(SE_RED_BLOCKS), 0, s, part, red);
}

namespace {

void real_cutoff_bins(const se_plan* p, int Ra[3])
{
    for (int d = 0; d < 3; d++) Ra[d] = (int)std::ceil(p->par.rc / p->g.h[d]) + 1;
}

// Shape of the blocked real-space sum: TB^3 target bins per block (about 48
// targets, or the plan's launch-shape knob); false when a block's candidate
// rows or target rows overflow the kernel's staging, which leaves the
// per-target kernel.
bool real2_shape(const se_plan* p, const int Ra[3], se_real2_geom* bg)
{
    const se_grid_geom& g = p->g;
    const int64_t nbins = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
    const double per_bin = (double)p->nt / (double)nbins;
    int TB = (int)std::lround(std::cbrt(48.0 / std::max(per_bin, 1e-9)));
    if (p->shape_real_tb > 0) TB = p->shape_real_tb;
    TB = std::max(1, std::min(TB, 4));
    bg->TB = TB;
    int span[3];
    for (int d = 0; d < 3; d++) {
        bg->nbk[d] = (g.nb[d] + TB - 1) / TB;
        span[d] = (TB * g.B[d] + 2 * Ra[d]) / g.B[d] + 2;
        if (!g.periodic[d]) span[d] = std::min(span[d], g.nb[d]);
    }
    bg->nblk = (int64_t)bg->nbk[0] * bg->nbk[1] * bg->nbk[2];
    bg->work = p->d_rwork;
    const int nseg = g.periodic[0] ? (span[0] + g.nb[0] - 1) / g.nb[0] + 1 : 1;
    return (int64_t)span[1] * span[2] * nseg <= SE_R2_SLOTS && TB * TB <= SE_R2_TROWS;
}

}  // namespace

void se_launch_scan_excl(int* v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, v, n);
}

void se_launch_real_prep(const se_plan* p, hipStream_t s)
{
    int Ra[3];
    real_cutoff_bins(p, Ra);
    se_real2_geom bg;
    if (!real2_shape(p, Ra, &bg)) return;
    se_real_args a{};
    a.g = p->g;
    a.tstart = p->tas ? p->d_src_start : p->d_tgt_start;
    hipLaunchKernelGGL(k_real2_chunks, dim3(grid1d(bg.nblk, 256)), dim3(256), 0, s, a, bg, p->d_rwork);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, p->d_rwork, bg.nblk);
}

void se_launch_real_space(const se_plan* p, int slot0, int nslot, hipStream_t s)
{
    se_real_args a;
    a.g = p->g;
    a.xt = (const double4*)(p->tas ? p->d_pos4 : p->d_tpos4);
    a.nt = p->nt;
    a.xs = (const double4*)p->d_pos4;
    a.ns = p->ns;
    a.f = (const double4*)se_slot_str4(p, slot0);
    a.nrm = (const double4*)p->d_nrm4;
    a.rtab = p->d_rtab;
    a.start = p->d_src_start;
    a.tstart = p->tas ? p->d_src_start : p->d_tgt_start;
    a.xi = p->par.xi;
    a.rc2 = p->par.rc * p->par.rc;
    a.rscale = SE_RTAB_N / se_rtab_xmax(p->par);
    real_cutoff_bins(p, a.Ra);
    a.tas = p->tas ? 1 : 0;
    a.u = se_slot_uR(p, slot0);
    a.flags = p->d_flags;
    se_real2_geom bg;
    if (real2_shape(p, a.Ra, &bg)) {
        const unsigned nwg = (unsigned)std::max<int64_t>(8, (bg.nblk + (p->nt + 63) / 64 + 3) / 4);
        if (nslot == 2 && p->kernel == SE_STOKESLET)
            hipLaunchKernelGGL((k_real2<SE_STOKESLET, 2>), dim3(nwg), dim3(256), 0, s, a, bg);
        else if (nslot == 2 && p->kernel == SE_ROTLET)
            hipLaunchKernelGGL((k_real2<SE_ROTLET, 2>), dim3(nwg), dim3(256), 0, s, a, bg);
        else if (nslot == 2 && p->kernel == SE_HARMONIC)
            hipLaunchKernelGGL((k_real2<SE_HARMONIC, 2>), dim3(nwg), dim3(256), 0, s, a, bg);
        else {
            for (int k = 0; k < nslot; k++) {
                se_real_args b = a;
                b.f = (const double4*)se_slot_str4(p, slot0 + k);
                b.u = se_slot_uR(p, slot0 + k);
                if (p->kernel == SE_STOKESLET)
                    hipLaunchKernelGGL((k_real2<SE_STOKESLET, 1>), dim3(nwg), dim3(256), 0, s, b, bg);
                else if (p->kernel == SE_ROTLET)
                    hipLaunchKernelGGL((k_real2<SE_ROTLET, 1>), dim3(nwg), dim3(256), 0, s, b, bg);
                else if (p->kernel == SE_HARMONIC)
                    hipLaunchKernelGGL((k_real2<SE_HARMONIC, 1>), dim3(nwg), dim3(256), 0, s, b, bg);
                else
                    hipLaunchKernelGGL((k_real2<SE_STRESSLET, 1>), dim3(nwg), dim3(256), 0, s, b, bg);
            }
        }
        return;
    }
    unsigned nb = (unsigned)std::min<int64_t>((p->nt + 3) / 4, SE_REAL_BLOCKS);
    for (int k = 0; k < nslot; k++) {
        se_real_args b = a;
        b.f = (const double4*)se_slot_str4(p, slot0 + k);
        b.u = se_slot_uR(p, slot0 + k);
        if (p->kernel == SE_STOKESLET) hipLaunchKernelGGL(k_real<SE_STOKESLET>, dim3(nb), dim3(256), 0, s, b);
        else if (p->kernel == SE_ROTLET) hipLaunchKernelGGL(k_real<SE_ROTLET>, dim3(nb), dim3(256), 0, s, b);
        else if (p->kernel == SE_HARMONIC) hipLaunchKernelGGL(k_real<SE_HARMONIC>, dim3(nb), dim3(256), 0, s, b);
        else hipLaunchKernelGGL(k_real<SE_STRESSLET>, dim3(nb), dim3(256), 0, s, b);
    }
}

void se_launch_finalize(const se_plan* p, int slot, double* u, double* u_real, double* u_fourier, hipStream_t s)
{
    se_fin_args a;
    a.nt = p->nt;
    a.perm = p->tas ? p->d_src_perm : p->d_tgt_perm;
    a.uF = se_slot_uF(p, slot);
    a.uR = se_slot_uR(p, slot);
    a.f64 = se_slot_fs64(p, slot);
    a.xt = p->tas ? p->d_src : p->d_tgt;
    a.red = se_slot_red(p, slot);
    // self terms (targets are sources): -4 xi/sqrt(pi) f (stokeslet), and
    // -2 xi/sqrt(pi) q for the harmonic (the limit of H - H^R at r = 0)
    a.self_c = 0.0;
    if (p->tas && p->kernel == SE_STOKESLET) a.self_c = -4.0 * p->par.xi / kSqrtPi;
    if (p->tas && p->kernel == SE_HARMONIC) a.self_c = -2.0 * p->par.xi / kSqrtPi;
    a.k0_c = (p->kernel == SE_STRESSLET && p->D == 3) ? -8.0 * M_PI / (p->g.L[0] * p->g.L[1] * p->g.L[2]) : 0.0;
    // D = 0 stokeslet: the optimal biharmonic b_B = -1/(2R) adds 4 b_B sum f
    // (eq. 0p-stokeslet-extra-contribution); remove it so u decays at infinity.
    for (int j = 0; j < 3; j++) a.gauge[j] = 0.0;
    if (p->D == 0 && p->kernel == SE_STOKESLET)
        for (int j = 0; j < 3; j++) a.gauge[j] = 2.0 / p->par.R;
    if (p->D == 3 && p->kernel == SE_HARMONIC) {
        // uniform neutralising background per charge set (the k -> 0 limit of
        // (4 pi/k^2)(gammaE - 1) / V): -pi / (V xi^2) sum q
        for (int j = 0; j < 3; j++)
            a.gauge[j] = -M_PI / (p->g.L[0] * p->g.L[1] * p->g.L[2] * p->par.xi * p->par.xi);
    }
    if (p->D == 1 && p->kernel == SE_HARMONIC) {
        // Hhat_R^{1P} is the transform of -2 log(rho/R) on rho < R (l_H = R);
        // return to l_H = 1: subtract (2 log R / L1) sum q per component
        for (int j = 0; j < 3; j++) a.gauge[j] = -2.0 * std::log(p->par.R) / p->g.L[0];
    }
    if (p->D == 1 && p->kernel == SE_STOKESLET) {
        // eq. (1p-stokeslet-extra-contribution) for l_H = R, l_B = R sqrt(e),
        // removed so that the result is in the gauge l_B = 1, l_H = 1/e
        const double lr = std::log(p->par.R);
        a.gauge[0] = -4.0 * (lr + 1.0) / p->g.L[0];
        a.gauge[1] = a.gauge[2] = -(2.0 * lr + 1.0) / p->g.L[0];
    }
    a.u = u;
    a.u_real = u_real;
    a.u_four = u_fourier;
    hipLaunchKernelGGL(k_finalize, dim3(grid1d(p->nt, 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// Jobs of merged batches: the blocked real-space sum of one plan (one job per
// pair of slots that a kernel takes together, else per slot), as
// se_launch_real_space launches it.  Variant: kernel type | RB << 3.
bool se_real_jobs(const se_plan* p, int nslot, std::vector<se_job>* out)
{
    se_real_job J;
    se_real_args& a = J.a;
    a.g = p->g;
    a.xt = (const double4*)(p->tas ? p->d_pos4 : p->d_tpos4);
    a.nt = p->nt;
    a.xs = (const double4*)p->d_pos4;
    a.ns = p->ns;
    a.nrm = (const double4*)p->d_nrm4;
    a.rtab = p->d_rtab;
    a.start = p->d_src_start;
    a.tstart = p->tas ? p->d_src_start : p->d_tgt_start;
    a.xi = p->par.xi;
    a.rc2 = p->par.rc * p->par.rc;
    a.rscale = SE_RTAB_N / se_rtab_xmax(p->par);
    real_cutoff_bins(p, a.Ra);
    a.tas = p->tas ? 1 : 0;
    a.flags = p->d_flags;
    if (!real2_shape(p, a.Ra, &J.bg)) return false;
    const int blocks = (int)std::max<int64_t>(1, (J.bg.nblk + (p->nt + 63) / 64 + 3) / 4);
    auto add = [&](int slot, int rb) {
        se_job j;
        j.family = SE_JOB_REAL;
        j.variant = p->kernel | (rb << 3);
        j.blocks = blocks;
        a.f = (const double4*)se_slot_str4(p, slot);
        a.u = se_slot_uR(p, slot);
        j.args.resize(sizeof(se_real_job));
        std::memcpy(j.args.data(), &J, sizeof(J));
        out->push_back(std::move(j));
    };
    if (nslot == 2 && p->kernel != SE_STRESSLET) add(0, 2);
    else
        for (int k = 0; k < nslot; k++) add(k, 1);
    return true;
}

int se_real_job_max() { return kRealJobMax; }

void se_real_launch_multi(int variant, const void* args, int n, int blocks, hipStream_t s)
{
    if (n <= 0 || n > kRealJobMax) return;
    const unsigned nwg = (unsigned)std::max(8, blocks);
    const se_real_job* jv = (const se_real_job*)args;
    const int ker = variant & 7, rb = variant >> 3;
    if (rb == 2) {
        if (ker == SE_STOKESLET) hipLaunchKernelGGL((k_real2_multi<SE_STOKESLET, 2>), dim3(nwg), dim3(256), 0, s, jv, n);
        else if (ker == SE_ROTLET) hipLaunchKernelGGL((k_real2_multi<SE_ROTLET, 2>), dim3(nwg), dim3(256), 0, s, jv, n);
        else hipLaunchKernelGGL((k_real2_multi<SE_HARMONIC, 2>), dim3(nwg), dim3(256), 0, s, jv, n);
    } else {
        if (ker == SE_STOKESLET) hipLaunchKernelGGL((k_real2_multi<SE_STOKESLET, 1>), dim3(nwg), dim3(256), 0, s, jv, n);
        else if (ker == SE_ROTLET) hipLaunchKernelGGL((k_real2_multi<SE_ROTLET, 1>), dim3(nwg), dim3(256), 0, s, jv, n);
        else if (ker == SE_HARMONIC)
            hipLaunchKernelGGL((k_real2_multi<SE_HARMONIC, 1>), dim3(nwg), dim3(256), 0, s, jv, n);
        else hipLaunchKernelGGL((k_real2_multi<SE_STRESSLET, 1>), dim3(nwg), dim3(256), 0, s, jv, n);
    }
}
