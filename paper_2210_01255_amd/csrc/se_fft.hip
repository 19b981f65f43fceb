// se_fft.hip -- FFT / scaling / IFFT steps (Sec. 3.2 steps (ii)-(iv)).
//
// Hand-written mixed-radix (2,3,4,5,7,8) Stockham transforms on LDS-resident
// lines, five passes over HBM per solve:
//   x  : real-to-complex along x (length-N/2 complex FFT + split), zero padded
//        input, writes the half spectrum [c][z][y][0..N/2];
//   y  : complex along y for bundles of adjacent kx columns (coalesced rows);
//   z  : complex along z, scaling (Green's function x screening / window^2)
//        and the inverse along z fused in one kernel, all components of a
//        column bundle resident in LDS;
//   y^-1, x^-1 (complex-to-real, truncated to the valid grid).
// The scaling includes the normalisation h^3/(N1 N2 N3) of the trapezoid
// rule in steps (ii), (iv) and (v), so the gathered sum is the Fourier part.
#include <algorithm>
#include <cstring>

#include "se_device.h"

namespace {

#define SE_MAX_RAD 24

struct se_fft_args {
    int Mg[3];
    int N[3];
    int Hx;     // half-spectrum extent along x (kx = 0 .. Hx-1)
    int Hp;     // row pitch of the half spectrum (complex elements, >= Hx)
    int ncomp;
    void* grid;
    void* spec;
    const double* tw;
    int tw_xh, tw_xp, tw_y, tw_z;
    uint64_t rad_xh, rad_y, rad_z;  // radix sequences, 4 bits per stage (first stage lowest)
    int nrad_xh, nrad_y, nrad_z;
    int lines;  // rows per workgroup (x passes)
    int cols;   // kx columns per workgroup (y, z passes)
    int cols_cap;  // upper bound on cols (0: automatic)
    // scaling
    int kernel;
    int D;
    double kfac[3];  // 2 pi / (h_i N_i)
    double xi;
    double inv4xi2;  // 1 / (4 xi^2)
    double scale;    // h1 h2 h3 / (N1 N2 N3)
    const double* invw2;  // 1/what0^2: [Hx | N1 | N2] per axis
    int iw_off[3];
    const double* ktab;   // D = 0: precomputed truncated kernel on the half spectrum [z][y][x]
    int skip_kx, skip_ky; // D = 1, 2: main-grid modes handled by an upsampled class
};

template <typename R>
using C = se_cplx<R>;

// ---------------------------------------------------------------- butterflies
// forward (dir = +1): out[k] = sum_n v[n] e^{-2 pi i n k / RAD}; inverse with +i
template <typename R>
__device__ __forceinline__ C<R> mul_mi(C<R> a, int dir)  // a * (-i dir)
{
    return dir > 0 ? C<R>{a.y, -a.x} : C<R>{-a.y, a.x};
}
template <typename R>
__device__ __forceinline__ C<R> cadd(C<R> a, C<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C<R> csub(C<R> a, C<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C<R> cscale(C<R> a, R s) { return {a.x * s, a.y * s}; }

template <typename R, int RAD>
__device__ __forceinline__ void dft_small(C<R>* v, int dir)
{
    if constexpr (RAD == 2) {
        C<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (RAD == 3) {
        const R s3 = (R)0.8660254037844386467637232;  // sin(2 pi/3)
        C<R> t1 = cadd(v[1], v[2]);
        C<R> t2 = csub(v[0], cscale(t1, (R)0.5));
        C<R> t3 = mul_mi(cscale(csub(v[1], v[2]), s3), dir);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, t3);
        v[2] = csub(t2, t3);
    } else if constexpr (RAD == 4) {
        C<R> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        C<R> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
        C<R> t = mul_mi(d13, dir);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, t);
        v[3] = csub(d02, t);
    } else if constexpr (RAD == 5) {
        const R c1 = (R)0.3090169943749474241022934, c2 = (R)-0.8090169943749474241022934;  // cos(2pi/5), cos(4pi/5)
        const R s1 = (R)0.9510565162951535721164393, s2 = (R)0.5877852522924731291687060;   // sin(2pi/5), sin(4pi/5)
        C<R> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        C<R> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        C<R> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
        C<R> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
        C<R> b1 = mul_mi(C<R>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y}, dir);
        C<R> b2 = mul_mi(C<R>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y}, dir);
        v[0] = {v[0].x + t1.x + t2.x, v[0].y + t1.y + t2.y};
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else if constexpr (RAD == 7) {
        // pairs (n, 7 - n): y_k = x0 + sum_n [cos(2 pi n k/7)(x_n + x_{7-n})
        //                               - i dir sin(2 pi n k/7)(x_n - x_{7-n})]
        const R cc[3] = {(R)0.6234898018587335305250049, (R)-0.2225209339563144042889026,
                         (R)-0.9009688679024191262361023};
        const R ss[3] = {(R)0.7818314824680298087084445, (R)0.9749279121818236070181317,
                         (R)0.4338837391175581204757683};
        C<R> sp[3], sm[3];
#pragma unroll
        for (int n = 0; n < 3; n++) {
            sp[n] = cadd(v[n + 1], v[6 - n]);
            sm[n] = csub(v[n + 1], v[6 - n]);
        }
        C<R> y[7];
        y[0] = {v[0].x + sp[0].x + sp[1].x + sp[2].x, v[0].y + sp[0].y + sp[1].y + sp[2].y};
#pragma unroll
        for (int k = 1; k <= 3; k++) {
            C<R> a = v[0], b = {(R)0, (R)0};
#pragma unroll
            for (int n = 1; n <= 3; n++) {
                const int m = (n * k) % 7;  // cos(2 pi m/7), sin(2 pi m/7) from the first half
                const R c = m <= 3 ? cc[m - 1] : cc[7 - m - 1];
                const R sn = m <= 3 ? ss[m - 1] : -ss[7 - m - 1];
                a = {a.x + c * sp[n - 1].x, a.y + c * sp[n - 1].y};
                b = {b.x + sn * sm[n - 1].x, b.y + sn * sm[n - 1].y};
            }
            C<R> t = mul_mi(b, dir);
            y[k] = cadd(a, t);
            y[7 - k] = csub(a, t);
        }
#pragma unroll
        for (int k = 0; k < 7; k++) v[k] = y[k];
    } else {
        C<R> e[4] = {v[0], v[2], v[4], v[6]};
        C<R> o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<R, 4>(e, dir);
        dft_small<R, 4>(o, dir);
        const R h = (R)0.7071067811865475244008444;
        C<R> w1 = {h, dir > 0 ? -h : h};
        C<R> w3 = {-h, dir > 0 ? -h : h};
        C<R> o1 = cmul(o[1], w1);
        C<R> o2 = mul_mi(o[2], dir);
        C<R> o3 = cmul(o[3], w3);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
}

// Division by a divisor d that is the same for the whole workgroup:
// q = floor(a m / 2^32) with m = floor((2^32 - 1)/d) + 1 (m = 0 stands for
// d = 1).  m - 2^32/d lies in (0, 1], so the quotient is exact while
// a < 2^32/d; the line kernels divide indices below 2^12 by divisors below
// 2^12.  The remainder uses 24-bit products (operands below 2^16).
struct se_udiv {
    int d;
    uint32_t m;
};

__device__ __forceinline__ se_udiv make_udiv(int d)
{
    return {d, d > 1 ? 0xFFFFFFFFu / (uint32_t)d + 1u : 0u};
}

__device__ __forceinline__ int udiv(int a, se_udiv u, int* rem)
{
    const int q = u.m ? (int)__umulhi((uint32_t)a, u.m) : a;
    *rem = a - __mul24(q, u.d);
    return q;
}

// Element loop i = threadIdx.x, + SE_FFT_THREADS, ... < n between HBM and
// LDS: each work item reads kCopyBatch elements (ld) before it writes any of
// them (st), so that many loads per work item are in flight at once; a plain
// strided loop waits for each element before it issues the next load.  The
// reads are unconditional (indices past the end read element n - 1 again),
// which keeps them in one branch-free block; ld must accept any i < n.
constexpr int kCopyBatch = 8;
template <typename Ld, typename St>
__device__ __forceinline__ void copy_batched(int n, Ld ld, St st)
{
    for (int i0 = threadIdx.x; i0 < n; i0 += kCopyBatch * SE_FFT_THREADS) {
        decltype(ld(0)) t[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; u++) t[u] = ld(min(i0 + u * SE_FFT_THREADS, n - 1));
#pragma unroll
        for (int u = 0; u < kCopyBatch; u++) {
            const int i = i0 + u * SE_FFT_THREADS;
            if (i < n) st(i, t[u]);
        }
    }
}

// Elements (lines x length) of one in-place transform call: each work item
// then holds at most ceil(E / RAD / SE_FFT_THREADS) butterflies.  Passes whose
// lines are longer than kIpElems use kernels built for kIpElemsLong, the
// longest line a plan admits; the smaller budget keeps the common kernels at
// fewer registers.
constexpr int kIpElems = 1536;
// elements between the column sets of the fused z pass beyond their size:
// with sets a multiple of 8 elements (128 bytes) apart, the lanes that read
// the same element of two components hit the same LDS banks
constexpr int kZSetPad = 4;
constexpr int kIpElemsLong = SE_FFT_LDS_ELEMS;
static_assert(kIpElems <= kIpElemsLong, "element budgets");

template <int RAD, int E = kIpElems>
constexpr int ip_per_thread()
{
    return (E / RAD + SE_FFT_THREADS - 1) / SE_FFT_THREADS;
}

// One Stockham stage of radix RAD over `nl` lines of length N held in LDS,
// in place: every work item reads the inputs of its butterflies (at most
// ip_per_thread<RAD>, in registers) and transforms them, the workgroup
// synchronises, and the results are written back over the inputs.  Line l
// starts at (l / lpg) * gs + (l % lpg) * ls, element e at + e * es.  With
// lines_fastest the line index varies fastest across work items, otherwise the
// butterfly index does (unit stride in LDS either way for the layouts used).
// One buffer per line instead of a ping-pong pair: twice the lines fit the
// LDS, so each barrier covers twice the butterflies.
template <typename R, int RAD, int DIR, int E = kIpElems>
__device__ __forceinline__ void stage_ip(C<R>* buf, int off, int N, int nl, int gs, int ls, int es, bool lines_fastest,
                                         const C<R>* tw, int Ns, se_udiv dnl, se_udiv dlpg)
{
    constexpr int K = ip_per_thread<RAD, E>();
    const int nb = N / RAD;
    const int total = nb * nl;
    const se_udiv dnb = make_udiv(nb), dns = make_udiv(Ns);
    const int istep = nb * es;  // between the inputs of one butterfly
    const int ostep = Ns * es;  // between its outputs
    C<R> v[K][RAD];
    int ob[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int idx = (int)threadIdx.x + k * SE_FFT_THREADS;
        ob[k] = -1;
        if (idx < total) {
            int line, j;
            if (lines_fastest) j = udiv(idx, dnl, &line);
            else line = udiv(idx, dnb, &j);
            int lr;
            const int lq = udiv(line, dlpg, &lr);
            const int base = off + __mul24(lq, gs) + __mul24(lr, ls);
            int jn;
            const int jq = udiv(j, dns, &jn);
            // this stage's twiddles w^{r jn} (w = e^{-2 pi i/(Ns RAD)}), r-major
            // from element Ns - 1 of the table: consecutive work items read
            // consecutive elements
            const int tb = Ns - 1 + jn;
            const int i0 = base + __mul24(j, es);
            v[k][0] = buf[i0];
#pragma unroll
            for (int r = 1; r < RAD; r++) {
                C<R> w = tw[tb + (r - 1) * Ns];
                if (DIR < 0) w.y = -w.y;
                v[k][r] = cmul(buf[i0 + r * istep], w);
            }
            dft_small<R, RAD>(v[k], DIR);
            ob[k] = base + __mul24(__mul24(jq, Ns) * RAD + jn, es);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (ob[k] >= 0) {
#pragma unroll
            for (int r = 0; r < RAD; r++) buf[ob[k] + r * ostep] = v[k][r];
        }
    }
    __syncthreads();
}

// Full in-place transform of nl lines (N * nl <= E) in direction DIR (+1:
// e^{-2 pi i n k/N}).  Line l starts at off + (l / lpg) * gs + (l % lpg) *
// ls, element e at + e * es.  The input must be complete (synchronised) on
// entry; the result is synchronised on return.
template <typename R, int DIR, int E = kIpElems>
__device__ __forceinline__ void fft_ip(C<R>* buf, int off, int N, int nl, int lpg, int gs, int ls, int es,
                                       bool lines_fastest, const C<R>* tw, const int* rad, int nrad)
{
    const se_udiv dnl = make_udiv(nl), dlpg = make_udiv(lpg);
    int Ns = 1;
    for (int s = 0; s < nrad; s++) {
        const int r = rad[s];
        switch (r) {
            case 2: stage_ip<R, 2, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
            case 3: stage_ip<R, 3, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
            case 4: stage_ip<R, 4, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
            case 5: stage_ip<R, 5, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
            case 7: stage_ip<R, 7, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
            default: stage_ip<R, 8, DIR, E>(buf, off, N, nl, gs, ls, es, lines_fastest, tw, Ns, dnl, dlpg); break;
        }
        Ns *= r;
    }
}

// radix sequence (4 bits per stage) into an LDS array
__device__ __forceinline__ void load_rad(int* dst, uint64_t code, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = (int)((code >> (4 * threadIdx.x)) & 15u);
}

template <typename R>
__device__ __forceinline__ void load_tw(C<R>* dst, const double* src, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = {(R)src[2 * i], (R)src[2 * i + 1]};
}

// ------------------------------------------------------------ x: real -> half
// Rows of M0 reals (zero padded to N0) as N0/2 complex values, one FFT of
// length N0/2, then the split into the half spectrum k = 0..N0/2.
template <typename R, int E>
__device__ __forceinline__ void fft_x_r2c_body(const se_fft_args& a, int blk)
{
    extern __shared__ double smem_d[];
    __shared__ int s_rad[16];
    load_rad(s_rad, a.rad_xh, a.nrad_xh);
    const int Nh = a.N[0] / 2;
    C<R>* tw = (C<R>*)smem_d;
    C<R>* twp = tw + Nh;
    C<R>* b0 = twp + Nh + 1;
    load_tw(tw, a.tw + 2 * a.tw_xh, Nh);
    load_tw(twp, a.tw + 2 * a.tw_xp, Nh + 1);
    const int64_t rows = (int64_t)a.ncomp * a.Mg[2] * a.Mg[1];
    const int64_t row0 = (int64_t)blk * a.lines;
    const int nl = (int)min((int64_t)a.lines, rows - row0);
    const R* grid = (const R*)a.grid;
    C<R>* spec = (C<R>*)a.spec;
    const int M0 = a.Mg[0];
    const se_udiv dNh = make_udiv(Nh), dNh1 = make_udiv(Nh + 1), dMy = make_udiv(a.Mg[1]);
    // (c z, y) of the block's first row; rows l < nl follow it
    const int64_t cz0 = row0 / a.Mg[1];
    const int y0 = (int)(row0 - cz0 * a.Mg[1]);
    // element i = l Nh + k of the block; with M0 even every pair (2k, 2k+1)
    // is one aligned complex element of the row (or past its end)
    if ((M0 & 1) == 0) {
        copy_batched(
            nl * Nh,
            [&](int i) {
                int k;
                const int l = udiv(i, dNh, &k);
                const C<R>* row = (const C<R>*)(grid + (row0 + l) * M0);
                const C<R> t = row[2 * k < M0 ? k : 0];
                return 2 * k < M0 ? t : C<R>{(R)0, (R)0};
            },
            [&](int i, C<R> v) { b0[i] = v; });
    } else {
        copy_batched(
            nl * Nh,
            [&](int i) {
                int k;
                const int l = udiv(i, dNh, &k);
                const R* row = grid + (row0 + l) * M0;
                const R re = (2 * k < M0) ? row[2 * k] : (R)0;
                const R im = (2 * k + 1 < M0) ? row[2 * k + 1] : (R)0;
                return C<R>{re, im};
            },
            [&](int i, C<R> v) { b0[i] = v; });
    }
    __syncthreads();
    fft_ip<R, 1, E>(b0, 0, Nh, nl, nl, 0, Nh, 1, false, tw, s_rad, a.nrad_xh);
    const C<R>* Z = b0;
    for (int i = threadIdx.x; i < nl * (Nh + 1); i += blockDim.x) {
        int k;
        const int l = udiv(i, dNh1, &k);
        C<R> zk = Z[l * Nh + (k == Nh ? 0 : k)];
        C<R> zn = Z[l * Nh + (k == 0 ? 0 : Nh - k)];
        zn.y = -zn.y;  // conj(Z_{N-k})
        C<R> A = {(zk.x + zn.x) * (R)0.5, (zk.y + zn.y) * (R)0.5};
        C<R> Bm = {(zk.x - zn.x) * (R)0.5, (zk.y - zn.y) * (R)0.5};
        // X_k = A_k - i e^{-2 pi i k/N0} (Z_k - conj Z_{N-k})/2
        C<R> t = cmul(Bm, twp[k]);
        C<R> X = {A.x + t.y, A.y - t.x};
        int y;
        const int64_t cz = cz0 + udiv(y0 + l, dMy, &y);
        spec[(cz * a.N[1] + y) * a.Hp + k] = X;
    }
}

// ------------------------------------------------------------ x: half -> real
template <typename R, int E>
__device__ __forceinline__ void fft_x_c2r_body(const se_fft_args& a, int blk)
{
    extern __shared__ double smem_d[];
    __shared__ int s_rad[16];
    load_rad(s_rad, a.rad_xh, a.nrad_xh);
    const int Nh = a.N[0] / 2;
    C<R>* tw = (C<R>*)smem_d;
    C<R>* twp = tw + Nh;
    C<R>* b0 = twp + Nh + 1;
    load_tw(tw, a.tw + 2 * a.tw_xh, Nh);
    load_tw(twp, a.tw + 2 * a.tw_xp, Nh + 1);
    __syncthreads();
    const int64_t rows = (int64_t)a.ncomp * a.Mg[2] * a.Mg[1];
    const int64_t row0 = (int64_t)blk * a.lines;
    const int nl = (int)min((int64_t)a.lines, rows - row0);
    R* grid = (R*)a.grid;
    const C<R>* spec = (const C<R>*)a.spec;
    const se_udiv dNh = make_udiv(Nh), dMy = make_udiv(a.Mg[1]);
    const int64_t cz0 = row0 / a.Mg[1];
    const int y0 = (int)(row0 - cz0 * a.Mg[1]);
    // element i = l Nh + k of the block; ld returns X_k and conj(X_{N-k})
    struct pair_t {
        C<R> xk, xn;
    };
    copy_batched(
        nl * Nh,
        [&](int i) {
            int k, y;
            const int l = udiv(i, dNh, &k);
            const int64_t cz = cz0 + udiv(y0 + l, dMy, &y);
            const C<R>* X = spec + (cz * a.N[1] + y) * a.Hp;
            return pair_t{X[k], X[Nh - k]};
        },
        [&](int i, pair_t p) {
            int k;
            (void)udiv(i, dNh, &k);
            C<R> xk = p.xk, xn = p.xn;
            xn.y = -xn.y;  // conj(X_{N-k})
            C<R> Ap = {xk.x + xn.x, xk.y + xn.y};
            C<R> d = {xk.x - xn.x, xk.y - xn.y};
            C<R> w = twp[k];
            w.y = -w.y;  // e^{+2 pi i k/N0}
            C<R> Bp = cmul(d, w);
            b0[i] = {Ap.x - Bp.y, Ap.y + Bp.x};  // A' + i B'
        });
    __syncthreads();
    fft_ip<R, -1, E>(b0, 0, Nh, nl, nl, 0, Nh, 1, false, tw, s_rad, a.nrad_xh);
    const C<R>* Z = b0;
    const int M0 = a.Mg[0];
    copy_batched(
        nl * Nh, [&](int i) { return Z[i]; },
        [&](int i, C<R> z) {
            int k;
            const int l = udiv(i, dNh, &k);
            R* row = grid + (row0 + l) * M0;
            if ((M0 & 1) == 0) {
                // one aligned complex store per pair (2k, 2k+1)
                if (2 * k < M0) ((C<R>*)row)[k] = z;
            } else {
                if (2 * k < M0) row[2 * k] = z.x;
                if (2 * k + 1 < M0) row[2 * k + 1] = z.y;
            }
        });
}

// ------------------------------------------------------------ y: complex
// A bundle of `cols` adjacent kx columns (contiguous in a row) for one (c, z).
template <typename R, int E, int DIR>
__device__ __forceinline__ void fft_y_body(const se_fft_args& a, int bid)
{
    constexpr int dir = DIR;
    extern __shared__ double smem_d[];
    __shared__ int s_rad[16];
    load_rad(s_rad, a.rad_y, a.nrad_y);
    const int Ny = a.N[1];
    const int Cc = a.cols;
    C<R>* tw = (C<R>*)smem_d;
    C<R>* b0 = tw + Ny;
    load_tw(tw, a.tw + 2 * a.tw_y, Ny);
    const int nbx = (a.Hx + Cc - 1) / Cc;
    int bx = bid % nbx;
    int64_t cz = bid / nbx;  // c * Mz + z
    const int kx0 = bx * Cc;
    C<R>* spec = (C<R>*)a.spec;
    C<R>* base = spec + cz * (int64_t)Ny * a.Hp;
    const int n_in = dir > 0 ? a.Mg[1] : Ny;
    const int n_out = dir > 0 ? Ny : a.Mg[1];
    const se_udiv dC = make_udiv(Cc);
    // element i = y Cc + col
    copy_batched(
        Ny * Cc,
        [&](int i) {
            int col;
            const int y = udiv(i, dC, &col);
            const int kx = kx0 + col;
            // unconditional load from a valid address (kx0 < Hx), then select
            const bool ok = kx < a.Hx && y < n_in;
            const C<R> t = base[ok ? (int64_t)y * a.Hp + kx : (int64_t)kx0];
            return C<R>{ok ? t.x : (R)0, ok ? t.y : (R)0};
        },
        [&](int i, C<R> v) { b0[i] = v; });
    __syncthreads();
    fft_ip<R, DIR, E>(b0, 0, Ny, Cc, Cc, 0, 1, Cc, true, tw, s_rad, a.nrad_y);
    const C<R>* Z = b0;
    copy_batched(
        n_out * Cc, [&](int i) { return Z[i]; },
        [&](int i, C<R> v) {
            int col;
            const int y = udiv(i, dC, &col);
            const int kx = kx0 + col;
            if (kx < a.Hx) base[(int64_t)y * a.Hp + kx] = v;
        });
}

// ------------------------------------------------------------------ scaling
// Step (iii), eq. (SE-scaling-disc): multiply by Ghat_R(k) gammahat(k;xi) /
// what(k)^2 and the trapezoid/FFT normalisation h1 h2 h3/(N1 N2 N3).  With
// Ghat = Khat Ahat (eqs. diffop-rel-fourier-1..3) and the scalar Ahat the
// biharmonic Bhat (stokeslet, stresslet) or harmonic Hhat (rotlet):
//   S:     u = c (-k^2 F + k (k.F)),                      c = Bhat gH W
//   Omega: u = -i c (F x k),                              c = Hhat gE W
//   T:     u = i c (-k^2 (2 F k + k tr F) + 2 k (k^T F k)), c = Bhat gH W
// (F symmetric for T).  Ahat is -8 pi/k^4 or 4 pi/k^2 for D = 3 with the
// k = 0 mode set to zero (eq. mod-kernel-3p), and the precomputed truncated
// kernel Ahat_{R,tr} for D = 0 (Sec. 3.5).  Odd kernels are zero on Nyquist
// indices (the real part of a non-Hermitian mode).
template <int KER>
__device__ __forceinline__ double green_scalar(const se_fft_args& a, int ix, int iy, int iz, double k2)
{
    if (a.D == 0) return a.ktab[((int64_t)iz * a.N[1] + iy) * a.Hx + ix];
    if (k2 == 0.0) return 0.0;
    const double r = 1.0 / k2;
    return se_harmonic_based(KER) ? 4.0 * M_PI * r : -8.0 * M_PI * r * r;
}

// u = Khat(k) F with the scalar factor c = Ahat gammahat W already formed.
// nyq: bit d set when component d of k sits on a Nyquist index (+-pi/h alias
// to one grid mode).  The stokeslet's k k^T then takes the mean over both
// aliases, which keeps k_d k_l only when both or neither of d, l are Nyquist
// components; this makes the scaled spectrum Hermitian, so that the real
// inverse transform equals the real part of the complex one (a half
// spectrum that is not Hermitian on its kx = 0 and Nyquist planes would
// otherwise leak through the real x transform with the 1/what^2 gain).
template <typename R, int KER>
__device__ __forceinline__ void apply_green(double cd, const double* k, double k2, const C<R>* F, C<R>* U,
                                            int nyq = 0)
{
    const R kr[3] = {(R)k[0], (R)k[1], (R)k[2]};
    const R kk = (R)k2;
    const R c = (R)cd;
    if constexpr (KER == SE_STOKESLET) {
        C<R> kf = {(R)0, (R)0}, kn = {(R)0, (R)0};  // k.F over the regular / the Nyquist components
#pragma unroll
        for (int l = 0; l < 3; l++) {
            if ((nyq >> l) & 1) kn = {kn.x + kr[l] * F[l].x, kn.y + kr[l] * F[l].y};
            else kf = {kf.x + kr[l] * F[l].x, kf.y + kr[l] * F[l].y};
        }
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const C<R> p = ((nyq >> j) & 1) ? kn : kf;
            U[j] = {c * (kr[j] * p.x - kk * F[j].x), c * (kr[j] * p.y - kk * F[j].y)};
        }
    } else if constexpr (KER == SE_HARMONIC) {
#pragma unroll
        for (int j = 0; j < 3; j++) U[j] = {c * F[j].x, c * F[j].y};
    } else if constexpr (KER == SE_ROTLET) {
        C<R> w[3];  // F x k
        w[0] = {F[1].x * kr[2] - F[2].x * kr[1], F[1].y * kr[2] - F[2].y * kr[1]};
        w[1] = {F[2].x * kr[0] - F[0].x * kr[2], F[2].y * kr[0] - F[0].y * kr[2]};
        w[2] = {F[0].x * kr[1] - F[1].x * kr[0], F[0].y * kr[1] - F[1].y * kr[0]};
#pragma unroll
        for (int j = 0; j < 3; j++) U[j] = {c * w[j].y, -c * w[j].x};  // -i c w
    } else {
        // symmetric F: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz
        C<R> Fk[3];
        Fk[0] = {F[0].x * kr[0] + F[3].x * kr[1] + F[4].x * kr[2], F[0].y * kr[0] + F[3].y * kr[1] + F[4].y * kr[2]};
        Fk[1] = {F[3].x * kr[0] + F[1].x * kr[1] + F[5].x * kr[2], F[3].y * kr[0] + F[1].y * kr[1] + F[5].y * kr[2]};
        Fk[2] = {F[4].x * kr[0] + F[5].x * kr[1] + F[2].x * kr[2], F[4].y * kr[0] + F[5].y * kr[1] + F[2].y * kr[2]};
        C<R> tr = {F[0].x + F[1].x + F[2].x, F[0].y + F[1].y + F[2].y};
        C<R> kFk = {kr[0] * Fk[0].x + kr[1] * Fk[1].x + kr[2] * Fk[2].x,
                    kr[0] * Fk[0].y + kr[1] * Fk[1].y + kr[2] * Fk[2].y};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C<R> v = {2 * kr[j] * kFk.x - kk * (2 * Fk[j].x + kr[j] * tr.x),
                      2 * kr[j] * kFk.y - kk * (2 * Fk[j].y + kr[j] * tr.y)};
            U[j] = {-c * v.y, c * v.x};  // i c v
        }
    }
}

template <typename R, int KER, int NC>
__device__ __forceinline__ void scale_point(const se_fft_args& a, int ix, int iy, int iz, C<R>* F, C<R>* U)
{
    const int kb[3] = {ix, iy < a.N[1] / 2 ? iy : iy - a.N[1], iz < a.N[2] / 2 ? iz : iz - a.N[2]};
    const double k[3] = {a.kfac[0] * kb[0], a.kfac[1] * kb[1], a.kfac[2] * kb[2]};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const int nyqb = (2 * ix == a.N[0] ? 1 : 0) | (2 * iy == a.N[1] ? 2 : 0) | (2 * iz == a.N[2] ? 4 : 0);
    const bool nyq = nyqb != 0;
    // D = 2: columns |kx|, |ky| <= k*; D = 1: planes kx <= k* (upsampled classes)
    const bool moved = (a.D == 2 && ix <= a.skip_kx && kb[1] <= a.skip_ky && -kb[1] <= a.skip_ky) ||
                       (a.D == 1 && ix <= a.skip_kx);
    const double G = moved ? 0.0 : green_scalar<KER>(a, ix, iy, iz, k2);
    if (G == 0.0 || (se_odd_kernel(KER) && nyq)) {
        U[0] = U[1] = U[2] = {(R)0, (R)0};
        return;
    }
    const double e = k2 * a.inv4xi2;
    const double gE = exp(-e);
    const double iw = a.invw2[a.iw_off[0] + ix] * a.invw2[a.iw_off[1] + iy] * a.invw2[a.iw_off[2] + iz];
    const double W = a.scale * iw;
    const double screen = se_harmonic_based(KER) ? gE : gE * (1.0 + e);
    apply_green<R, KER>(G * screen * W, k, k2, F, U, nyqb);
}

// Plain complex transform along z (no scaling) for `ncomp` components.
template <typename R, int E, int DIR>
__global__ void __launch_bounds__(SE_FFT_THREADS) k_fft_z(se_fft_args a)
{
    constexpr int dir = DIR;
    extern __shared__ double smem_d[];
    __shared__ int s_rad[16];
    load_rad(s_rad, a.rad_z, a.nrad_z);
    const int Nz = a.N[2];
    const int Cc = a.cols;
    C<R>* tw = (C<R>*)smem_d;
    C<R>* b0 = tw + Nz;
    load_tw(tw, a.tw + 2 * a.tw_z, Nz);
    const int nbx = (a.Hx + Cc - 1) / Cc;
    const int blk = se_xcd_block(blockIdx.x, gridDim.x);
    const int bx = blk % nbx;
    const int rest = blk / nbx;
    const int y = rest % a.N[1];
    const int c = rest / a.N[1];
    const int kx0 = bx * Cc;
    const int Mz = a.Mg[2];
    const int64_t zstride = (int64_t)a.N[1] * a.Hp;
    C<R>* spec = (C<R>*)a.spec + (int64_t)c * Mz * zstride;
    const int n_in = dir > 0 ? Mz : Nz;
    const int n_out = dir > 0 ? Nz : Mz;
    const se_udiv dC = make_udiv(Cc);
    copy_batched(
        Nz * Cc,
        [&](int i) {
            int col;
            const int z = udiv(i, dC, &col);
            const int kx = kx0 + col;
            const bool ok = kx < a.Hx && z < n_in && z < Mz;
            const C<R> t = spec[ok ? z * zstride + (int64_t)y * a.Hp + kx : (int64_t)y * a.Hp + kx0];
            return C<R>{ok ? t.x : (R)0, ok ? t.y : (R)0};
        },
        [&](int i, C<R> v) { b0[i] = v; });
    __syncthreads();
    fft_ip<R, DIR, E>(b0, 0, Nz, Cc, Cc, 0, 1, Cc, true, tw, s_rad, a.nrad_z);
    const C<R>* Z = b0;
    copy_batched(
        n_out * Cc, [&](int i) { return Z[i]; },
        [&](int i, C<R> v) {
            int col;
            const int z = udiv(i, dC, &col);
            const int kx = kx0 + col;
            if (kx < a.Hx && z < Mz) spec[z * zstride + (int64_t)y * a.Hp + kx] = v;
        });
}

// Transform along z, scaling and inverse transform for one bundle of `cols`
// kx columns at one y, all components resident in LDS (NC column sets,
// transformed in place, several components per call).
template <typename R, int KER, int NC, int E>
__device__ __forceinline__ void fft_z_scale_body(const se_fft_args& a, int blk)
{
    extern __shared__ double smem_d[];
    __shared__ int s_rad[16];
    load_rad(s_rad, a.rad_z, a.nrad_z);
    const int Nz = a.N[2];
    const int Cc = a.cols;
    const int cs = Nz * Cc;          // LDS column-set size
    const int csp = cs + kZSetPad;   // column-set stride (bank offset between components)
    C<R>* tw = (C<R>*)smem_d;
    C<R>* sets = tw + Nz;
    load_tw(tw, a.tw + 2 * a.tw_z, Nz);
    const int nbx = (a.Hx + Cc - 1) / Cc;
    const int bx = blk % nbx;
    const int y = blk / nbx;
    const int kx0 = bx * Cc;
    const int Mz = a.Mg[2];
    const int64_t cstride = (int64_t)Mz * a.N[1] * a.Hp;
    const int64_t zstride = (int64_t)a.N[1] * a.Hp;
    C<R>* spec = (C<R>*)a.spec;
    const se_udiv dcs = make_udiv(cs), dC = make_udiv(Cc);
    copy_batched(
        NC * cs,
        [&](int i) {
            int rem, col;
            const int c = udiv(i, dcs, &rem);
            const int z = udiv(rem, dC, &col);
            const int kx = kx0 + col;
            const bool ok = kx < a.Hx && z < Mz;
            const C<R> t = spec[c * cstride + (ok ? z * zstride + (int64_t)y * a.Hp + kx : (int64_t)y * a.Hp + kx0)];
            return C<R>{ok ? t.x : (R)0, ok ? t.y : (R)0};
        },
        [&](int i, C<R> v) {
            int rem;
            const int c = udiv(i, dcs, &rem);
            sets[c * csp + rem] = v;
        });
    __syncthreads();
    // as many components per transform call as fit kIpElems (lines of one
    // component are Cc adjacent columns; components are cs apart)
    const int gc = max(1, min(NC, E / cs));
    for (int c0 = 0; c0 < NC; c0 += gc)
        fft_ip<R, 1, E>(sets, c0 * csp, Nz, min(gc, NC - c0) * Cc, Cc, csp, 1, Cc, true, tw, s_rad, a.nrad_z);
    for (int i = threadIdx.x; i < cs; i += blockDim.x) {
        int col;
        const int z = udiv(i, dC, &col);
        int kx = kx0 + col;
        if (kx >= a.Hx) continue;
        C<R> F[NC], U[3];
#pragma unroll
        for (int c = 0; c < NC; c++) F[c] = sets[c * csp + i];
        scale_point<R, KER, NC>(a, kx, y, z, F, U);
#pragma unroll
        for (int j = 0; j < 3; j++) sets[j * csp + i] = U[j];
    }
    __syncthreads();
    for (int c0 = 0; c0 < 3; c0 += gc)
        fft_ip<R, -1, E>(sets, c0 * csp, Nz, min(gc, 3 - c0) * Cc, Cc, csp, 1, Cc, true, tw, s_rad, a.nrad_z);
    copy_batched(
        3 * cs,
        [&](int i) {
            int rem;
            const int c = udiv(i, dcs, &rem);
            return sets[c * csp + rem];
        },
        [&](int i, C<R> v) {
            int rem, col;
            const int c = udiv(i, dcs, &rem);
            const int z = udiv(rem, dC, &col);
            const int kx = kx0 + col;
            if (kx < a.Hx && z < Mz) spec[c * cstride + z * zstride + (int64_t)y * a.Hp + kx] = v;
        });
}

// Kernels over one plan's pass (neighbouring blocks share an XCD and its
// L2) and merged kernels over the jobs of many plans: job j's record is
// av[j] and its blocks are boff[j] .. boff[j+1] - 1 of the launch.
__device__ __forceinline__ int fft_job_of(const int* __restrict__ boff, int n, int g)
{
    int lo = 0, hi = n;  // largest j with boff[j] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename R, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS, 4) k_fft_x_r2c(se_fft_args a)
{
    fft_x_r2c_body<R, E>(a, se_xcd_block(blockIdx.x, gridDim.x));
}
template <typename R, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS, 4) k_fft_x_r2c_multi(const se_fft_args* __restrict__ av,
                                                                     const int* __restrict__ boff, int n)
{
    const int g = se_xcd_block(blockIdx.x, gridDim.x), j = fft_job_of(boff, n, g);
    fft_x_r2c_body<R, E>(av[j], g - boff[j]);
}
template <typename R, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS, 4) k_fft_x_c2r(se_fft_args a)
{
    fft_x_c2r_body<R, E>(a, se_xcd_block(blockIdx.x, gridDim.x));
}
template <typename R, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS, 4) k_fft_x_c2r_multi(const se_fft_args* __restrict__ av,
                                                                     const int* __restrict__ boff, int n)
{
    const int g = se_xcd_block(blockIdx.x, gridDim.x), j = fft_job_of(boff, n, g);
    fft_x_c2r_body<R, E>(av[j], g - boff[j]);
}
template <typename R, int E, int DIR>
__global__ void __launch_bounds__(SE_FFT_THREADS, 5) k_fft_y(se_fft_args a)
{
    fft_y_body<R, E, DIR>(a, se_xcd_block(blockIdx.x, gridDim.x));
}
template <typename R, int E, int DIR>
__global__ void __launch_bounds__(SE_FFT_THREADS, 5) k_fft_y_multi(const se_fft_args* __restrict__ av,
                                                                 const int* __restrict__ boff, int n)
{
    const int g = se_xcd_block(blockIdx.x, gridDim.x), j = fft_job_of(boff, n, g);
    fft_y_body<R, E, DIR>(av[j], g - boff[j]);
}
template <typename R, int KER, int NC, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS) k_fft_z_scale(se_fft_args a)
{
    fft_z_scale_body<R, KER, NC, E>(a, se_xcd_block(blockIdx.x, gridDim.x));
}
template <typename R, int KER, int NC, int E>
__global__ void __launch_bounds__(SE_FFT_THREADS) k_fft_z_scale_multi(const se_fft_args* __restrict__ av,
                                                                    const int* __restrict__ boff, int n)
{
    const int g = se_xcd_block(blockIdx.x, gridDim.x), j = fft_job_of(boff, n, g);
    fft_z_scale_body<R, KER, NC, E>(av[j], g - boff[j]);
}

// LDS budgets (bytes) of the line kernels: two workgroups per CU.
constexpr size_t kFftLds = 80 * 1024;
constexpr size_t kFftLdsStatic = 256;  // static LDS of the line kernels (radix table), rounded up

// Radix sequence of a line length, in the stage order of se_fft_radix_order.
void set_radices(int n, uint64_t* dst, int* cnt)
{
    std::vector<int> r;
    se_fft_radix_order(n, &r);
    *cnt = (int)std::min<size_t>(r.size(), 16);
    uint64_t code = 0;
    for (int i = 0; i < *cnt; i++) code |= (uint64_t)r[i] << (4 * i);
    *dst = code;
}

se_fft_args make_fft_args_geom(const int* Mg, const int* N, const double* h, void* grid, void* spec,
                               const double* tw, const int* tw_off, int ncomp)
{
    se_fft_args a;
    std::memset(&a, 0, sizeof(a));
    for (int d = 0; d < 3; d++) {
        a.Mg[d] = Mg[d];
        a.N[d] = N[d];
    }
    a.Hx = N[0] / 2 + 1;
    a.Hp = a.Hx;
    a.ncomp = ncomp;
    a.grid = grid;
    a.spec = spec;
    a.tw = tw;
    a.tw_xh = tw_off[0];
    a.tw_xp = tw_off[1];
    a.tw_y = tw_off[2];
    a.tw_z = tw_off[3];
    set_radices(N[0] / 2, &a.rad_xh, &a.nrad_xh);
    set_radices(N[1], &a.rad_y, &a.nrad_y);
    set_radices(N[2], &a.rad_z, &a.nrad_z);
    double hv = 1.0, nv = 1.0;
    for (int d = 0; d < 3; d++) {
        a.kfac[d] = 2.0 * M_PI / (h[d] * N[d]);
        hv *= h[d];
        nv *= N[d];
    }
    a.scale = hv / nv;
    return a;
}

se_fft_args make_fft_args(const se_plan* p, int ncomp, int slot)
{
    se_fft_args a = make_fft_args_geom(p->g.Mg, p->Nfft, p->g.h, se_slot_grid(p, slot), se_slot_spec(p, slot), p->d_tw,
                                       p->tw_off, ncomp);
    a.Hp = p->Hp;
    a.cols_cap = p->shape_fft_cols;
    a.kernel = p->kernel;
    a.D = p->D;
    a.xi = p->par.xi;
    a.inv4xi2 = 1.0 / (4.0 * p->par.xi * p->par.xi);
    a.invw2 = p->d_invw2;
    a.iw_off[0] = 0;
    a.iw_off[1] = p->Hx;
    a.iw_off[2] = p->Hx + p->Nfft[1];
    a.ktab = p->d_ktab;
    a.skip_kx = -1;
    a.skip_ky = -1;
    if (p->D == 2) {
        a.skip_kx = p->cls[1].active ? p->cls[1].nkx - 1 : 0;
        a.skip_ky = p->cls[1].active ? (p->cls[1].ny - 1) / 2 : 0;
    } else if (p->D == 1) {
        a.skip_kx = p->cls[1].active ? p->cls[1].nkx : 0;
    }
    return a;
}

// element budget of the kernels for lines of length N
inline int ip_budget(int N) { return N > kIpElems ? kIpElemsLong : kIpElems; }

template <typename R>
int x_lines(int Nh)
{
    const int budget = (int)(kFftLds / sizeof(C<R>)) - (2 * Nh + 1);
    return std::max(1, std::min(budget / Nh, ip_budget(Nh) / Nh));
}

// columns per bundle for a pass holding `sets` column sets of length N plus
// the twiddles within the LDS budget, one set per in-place transform call
template <typename R>
int bundle_cols(int N, int sets, int cap = 16, int pad = 0)
{
    const int budget = (int)(kFftLds / sizeof(C<R>)) - N - sets * pad;
    int c = std::max(1, std::min({cap > 0 ? cap : 16, budget / (sets * N), ip_budget(N) / N}));
    while (c & (c - 1)) c &= c - 1;  // power of two
    return c;
}

template <typename K>
void allow_lds(K kern, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R>
void run_x_r2c(se_fft_args a, int ncomp, hipStream_t s)
{
    const int Nh = a.N[0] / 2;
    a.ncomp = ncomp;
    a.lines = x_lines<R>(Nh);
    int64_t rows = (int64_t)ncomp * a.Mg[2] * a.Mg[1];
    size_t lds = (size_t)(2 * Nh + 1 + a.lines * Nh) * sizeof(C<R>);
    auto kern = Nh > kIpElems ? k_fft_x_r2c<R, kIpElemsLong> : k_fft_x_r2c<R, kIpElems>;
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)((rows + a.lines - 1) / a.lines)), dim3(SE_FFT_THREADS), lds, s, a);
}

template <typename R>
void run_x_c2r(se_fft_args a, int ncomp, hipStream_t s)
{
    const int Nh = a.N[0] / 2;
    a.ncomp = ncomp;
    a.lines = x_lines<R>(Nh);
    int64_t rows = (int64_t)ncomp * a.Mg[2] * a.Mg[1];
    size_t lds = (size_t)(2 * Nh + 1 + a.lines * Nh) * sizeof(C<R>);
    auto kern = Nh > kIpElems ? k_fft_x_c2r<R, kIpElemsLong> : k_fft_x_c2r<R, kIpElems>;
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)((rows + a.lines - 1) / a.lines)), dim3(SE_FFT_THREADS), lds, s, a);
}

template <typename R>
void run_y(se_fft_args a, int ncomp, int dir, hipStream_t s)
{
    a.cols = bundle_cols<R>(a.N[1], 1, a.cols_cap);
    int nbx = (a.Hx + a.cols - 1) / a.cols;
    size_t lds = (size_t)(a.N[1] + a.cols * a.N[1]) * sizeof(C<R>);
    auto kern = dir > 0 ? (a.N[1] > kIpElems ? k_fft_y<R, kIpElemsLong, 1> : k_fft_y<R, kIpElems, 1>)
                        : (a.N[1] > kIpElems ? k_fft_y<R, kIpElemsLong, -1> : k_fft_y<R, kIpElems, -1>);
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)(nbx * ncomp * a.Mg[2])), dim3(SE_FFT_THREADS), lds, s, a);
}

template <typename R>
void run_z_plain(se_fft_args a, int ncomp, int dir, hipStream_t s)
{
    a.cols = bundle_cols<R>(a.N[2], 1, a.cols_cap);
    int nbx = (a.Hx + a.cols - 1) / a.cols;
    size_t lds = (size_t)(a.N[2] + a.cols * a.N[2]) * sizeof(C<R>);
    auto kern = dir > 0 ? (a.N[2] > kIpElems ? k_fft_z<R, kIpElemsLong, 1> : k_fft_z<R, kIpElems, 1>)
                        : (a.N[2] > kIpElems ? k_fft_z<R, kIpElemsLong, -1> : k_fft_z<R, kIpElems, -1>);
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)(nbx * a.N[1] * ncomp)), dim3(SE_FFT_THREADS), lds, s, a);
}

template <typename R>
void cls_gather(const se_plan* p, int slot, hipStream_t s);
template <typename R>
void cls_scatter(const se_plan* p, int slot, hipStream_t s);

template <typename R>
void launch_fwd(const se_plan* p, int slot, hipStream_t s)
{
    se_fft_args a = make_fft_args(p, p->ncomp, slot);
    run_x_r2c<R>(a, p->ncomp, s);
    if (p->D == 1) cls_gather<R>(p, slot, s);
    run_y<R>(a, p->ncomp, 1, s);
    if (p->D == 2) cls_gather<R>(p, slot, s);
}

template <typename R, int KER, int NC>
void launch_z(const se_plan* p, int slot, hipStream_t s)
{
    se_fft_args a = make_fft_args(p, NC, slot);
    // two columns by default: the components then share transform calls
    // (kIpElems / (2 N) of them per call), which shortens the chain of
    // barrier-separated stages per column more than wider rows would help
    a.cols = bundle_cols<R>(p->Nfft[2], NC, p->shape_fft_cols > 0 ? p->shape_fft_cols : 2, kZSetPad);
    int nbx = (p->Hx + a.cols - 1) / a.cols;
    size_t lds = (size_t)(p->Nfft[2] + NC * (a.cols * p->Nfft[2] + kZSetPad)) * sizeof(C<R>);
    auto kern = p->Nfft[2] > kIpElems ? k_fft_z_scale<R, KER, NC, kIpElemsLong> : k_fft_z_scale<R, KER, NC, kIpElems>;
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)(nbx * p->Nfft[1])), dim3(SE_FFT_THREADS), lds, s, a);
}

template <typename R>
void launch_inv(const se_plan* p, int slot, hipStream_t s)
{
    se_fft_args a = make_fft_args(p, 3, slot);
    run_y<R>(a, 3, -1, s);
    if (p->D == 1) cls_scatter<R>(p, slot, s);
    run_x_c2r<R>(a, 3, s);
}

template <typename R>
void launch_z_dispatch(const se_plan* p, int slot, hipStream_t s)
{
    if (p->kernel == SE_STOKESLET) launch_z<R, SE_STOKESLET, 3>(p, slot, s);
    else if (p->kernel == SE_ROTLET) launch_z<R, SE_ROTLET, 3>(p, slot, s);
    else if (p->kernel == SE_HARMONIC) launch_z<R, SE_HARMONIC, 3>(p, slot, s);
    else launch_z<R, SE_STRESSLET, 6>(p, slot, s);
}

// ------------------------------------------------- adaptive FFT: upsampled classes
// Sec. 3.4 (AFT): modes k^P = 0 and k^P in K_* are transformed along the free
// directions with upsampling s0 and s_* (zero padding in real space), scaled
// with the modified kernels (eqs. mod-stokeslet-2p .. mod-stresslet-2p,
// mod-rotlet-1p .. mod-stresslet-1p) or the regular ones, transformed back and
// truncated to the extended grid.
struct se_cls_args {
    int D;
    int zero;
    int nkx, ny, nz;
    int kx_lo, ky_lo;
    int Hp, N1, Mg1, Mz;  // main half spectrum [c][Mz][N1][Hp], valid y rows Mg1
    void* spec;
    void* buf;
    const double* kv;
    const double* iw;
    const double* mk;
    double xi, R, scale;
};

void* cls_slot_buf(const se_plan* p, const se_aft_class& c, int slot)
{
    return (char*)c.buf + (size_t)slot * p->ncomp * c.nkx * c.ny * c.nz * 2 * se_real_bytes(p);
}

se_cls_args make_cls_args(const se_plan* p, const se_aft_class& c, int slot)
{
    se_cls_args a;
    std::memset(&a, 0, sizeof(a));
    a.D = p->D;
    a.zero = c.zero;
    a.nkx = c.nkx;
    a.ny = c.ny;
    a.nz = c.nz;
    a.kx_lo = c.kx_lo;
    a.ky_lo = c.ky_lo;
    a.Hp = p->Hp;
    a.N1 = p->Nfft[1];
    a.Mg1 = p->g.Mg[1];
    a.Mz = p->g.Mg[2];
    a.spec = se_slot_spec(p, slot);
    a.buf = cls_slot_buf(p, c, slot);
    a.kv = c.kv;
    a.iw = c.iw;
    a.mk = c.mk;
    a.xi = p->par.xi;
    a.R = p->par.R;
    a.scale = c.scale;
    return a;
}

// main spectrum -> zero-padded class buffer (ncomp components)
template <typename R>
__global__ void k_cls_gather(se_cls_args a, int ncomp)
{
    const int64_t n = (int64_t)a.nkx * a.ny * a.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ncomp) return;
    const int c = (int)(i / n);
    const int64_t r = i - c * n;
    const int ix = (int)(r % a.nkx);
    const int iy = (int)((r / a.nkx) % a.ny);
    const int iz = (int)(r / ((int64_t)a.nkx * a.ny));
    const C<R>* spec = (const C<R>*)a.spec;
    C<R> v = {(R)0, (R)0};
    int y = -1;
    if (a.D == 2) y = (a.ky_lo + iy + a.N1) % a.N1;
    else if (iy < a.Mg1) y = iy;
    if (y >= 0 && iz < a.Mz) v = spec[(((int64_t)c * a.Mz + iz) * a.N1 + y) * a.Hp + a.kx_lo + ix];
    ((C<R>*)a.buf)[i] = v;
}

// class buffer (3 components) -> main spectrum, truncated to the extended grid
template <typename R>
__global__ void k_cls_scatter(se_cls_args a)
{
    const int rows = a.D == 2 ? a.ny : a.Mg1;
    const int64_t n = (int64_t)a.nkx * rows * a.Mz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    const int c = (int)(i / n);
    const int64_t r = i - c * n;
    const int ix = (int)(r % a.nkx);
    const int iy = (int)((r / a.nkx) % rows);
    const int iz = (int)(r / ((int64_t)a.nkx * rows));
    int y = iy;
    if (a.D == 2) {
        if (!a.zero && a.kx_lo + ix == 0 && a.ky_lo + iy == 0) return;  // owned by the k^P = 0 class
        y = (a.ky_lo + iy + a.N1) % a.N1;
    }
    const C<R>* buf = (const C<R>*)a.buf;
    ((C<R>*)a.spec)[(((int64_t)c * a.Mz + iz) * a.N1 + y) * a.Hp + a.kx_lo + ix] =
        buf[(((int64_t)c * a.nz + iz) * a.ny + iy) * a.nkx + ix];
}

template <typename R, int KER, int NC>
__global__ void k_cls_scale(se_cls_args a)
{
    const int64_t n = (int64_t)a.nkx * a.ny * a.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ix = (int)(i % a.nkx);
    const int iy = (int)((i / a.nkx) % a.ny);
    const int iz = (int)(i / ((int64_t)a.nkx * a.ny));
    C<R>* buf = (C<R>*)a.buf;
    C<R> F[NC], U[3];
#pragma unroll
    for (int c = 0; c < NC; c++) F[c] = buf[c * n + i];
    const double k[3] = {a.kv[ix], a.kv[a.nkx + iy], a.kv[a.nkx + a.ny + iz]};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const bool nyq = (2 * iz == a.nz) || (a.D == 1 && 2 * iy == a.ny);
    const double e = k2 / (4.0 * a.xi * a.xi);
    const double gE = exp(-e);
    const double screen = se_harmonic_based(KER) ? gE : gE * (1.0 + e);
    const double W = a.scale * a.iw[ix] * a.iw[a.nkx + iy] * a.iw[a.nkx + a.ny + iz];
    U[0] = U[1] = U[2] = {(R)0, (R)0};
    const bool kp0 = (k[0] == 0.0) && (a.D == 1 || k[1] == 0.0);
    if (se_odd_kernel(KER) && nyq) {
        // odd kernels: no Hermitian partner on Nyquist indices
    } else if (!a.zero) {
        if (!kp0) {
            const double G = se_harmonic_based(KER) ? 4.0 * M_PI / k2 : -8.0 * M_PI / (k2 * k2);
            apply_green<R, KER>(G * screen * W, k, k2, F, U);
        }
    } else if (a.D == 2) {
        const double kz = k[2], Rk = a.R * kz;
        if constexpr (KER == SE_HARMONIC) {
            // Hhat_R^{2P} per component, limit -2 pi R^2
            const double H = kz == 0.0 ? -2.0 * M_PI * a.R * a.R
                                       : 4.0 * M_PI / (kz * kz) * (1.0 - cos(Rk) - Rk * sin(Rk));
            const R c = (R)(H * screen * W);
#pragma unroll
            for (int j = 0; j < 3; j++) U[j] = {c * F[j].x, c * F[j].y};
        } else if constexpr (KER == SE_STOKESLET) {
            // Hhat_R^{2P} D^S, limit -2 pi R^2
            const double H = kz == 0.0 ? -2.0 * M_PI * a.R * a.R
                                       : 4.0 * M_PI / (kz * kz) * (1.0 - cos(Rk) - Rk * sin(Rk));
            const R c = (R)(2.0 * H * screen * W);
            U[0] = {c * F[0].x, c * F[0].y};
            U[1] = {c * F[1].x, c * F[1].y};
        } else {
            // Zhat_R^{2P} = -i z, z = 4 pi (1 - cos(R k3))/k3, limit 0
            const double z = kz == 0.0 ? 0.0 : 4.0 * M_PI * (1.0 - cos(Rk)) / kz;
            const R c = (R)(z * screen * W);
            if constexpr (KER == SE_ROTLET) {
                U[0] = {c * F[1].y, -c * F[1].x};   // -i c F_2
                U[1] = {-c * F[0].y, c * F[0].x};   // +i c F_1
            } else {
                // D^T: u1 = -4 Zhat F13, u2 = -4 Zhat F23, u3 = -2 Zhat tr F
                U[0] = {-4 * c * F[4].y, 4 * c * F[4].x};
                U[1] = {-4 * c * F[5].y, 4 * c * F[5].x};
                C<R> tr = {F[0].x + F[1].x + F[2].x, F[0].y + F[1].y + F[2].y};
                U[2] = {-2 * c * tr.y, 2 * c * tr.x};
            }
        }
    } else {
        const double H = a.mk[2 * (iz * (int64_t)a.ny + iy)];
        const double B = a.mk[2 * (iz * (int64_t)a.ny + iy) + 1];
        if constexpr (KER == SE_ROTLET || KER == SE_HARMONIC) {
            apply_green<R, KER>(H * screen * W, k, k2, F, U);
        } else if constexpr (KER == SE_STOKESLET) {
            apply_green<R, KER>(B * screen * W, k, k2, F, U);
            const R c = (R)(2.0 * H * screen * W);
            U[0] = {c * F[0].x, c * F[0].y};
        } else {
            const R cH = (R)(H * screen * W), cB = (R)(B * screen * W);
            const R k2r = (R)k[1], k3r = (R)k[2], kk = (R)k2;
            // 4 i cH (k2 F12 + k3 F13)
            C<R> t0 = {4 * cH * (k2r * F[3].x + k3r * F[4].x), 4 * cH * (k2r * F[3].y + k3r * F[4].y)};
            U[0] = {-t0.y, t0.x};
            const R a22 = k2r * (3 * kk - 2 * k2r * k2r), a23 = 2 * k3r * (kk - 2 * k2r * k2r),
                    a33 = k2r * (kk - 2 * k3r * k3r);
            const R b22 = k3r * (kk - 2 * k2r * k2r), b23 = 2 * k2r * (kk - 2 * k3r * k3r),
                    b33 = k3r * (3 * kk - 2 * k3r * k3r);
            C<R> t1 = {2 * cH * k2r * F[0].x - cB * (a22 * F[1].x + a23 * F[5].x + a33 * F[2].x),
                       2 * cH * k2r * F[0].y - cB * (a22 * F[1].y + a23 * F[5].y + a33 * F[2].y)};
            C<R> t2 = {2 * cH * k3r * F[0].x - cB * (b22 * F[1].x + b23 * F[5].x + b33 * F[2].x),
                       2 * cH * k3r * F[0].y - cB * (b22 * F[1].y + b23 * F[5].y + b33 * F[2].y)};
            U[1] = {-t1.y, t1.x};
            U[2] = {-t2.y, t2.x};
        }
    }
#pragma unroll
    for (int j = 0; j < 3; j++) buf[j * n + i] = U[j];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

se_fft_args cls_fft_args(const se_plan* p, const se_aft_class& c, int slot)
{
    const int Mg[3] = {2, c.ny, c.nz};
    const int N[3] = {2, c.ny, c.nz};
    se_fft_args a = make_fft_args_geom(Mg, N, p->g.h, nullptr, cls_slot_buf(p, c, slot), c.tw, c.tw_off, p->ncomp);
    a.Hx = c.nkx;
    a.Hp = c.nkx;
    a.cols_cap = p->shape_fft_cols;
    return a;
}

template <typename R>
void cls_gather(const se_plan* p, int slot, hipStream_t s)
{
    for (const se_aft_class& c : p->cls) {
        if (!c.active) continue;
        se_cls_args a = make_cls_args(p, c, slot);
        int64_t n = (int64_t)c.nkx * c.ny * c.nz * p->ncomp;
        hipLaunchKernelGGL(k_cls_gather<R>, dim3(nblk(n)), dim3(256), 0, s, a, p->ncomp);
    }
}

template <typename R>
void cls_scatter(const se_plan* p, int slot, hipStream_t s)
{
    for (const se_aft_class& c : p->cls) {
        if (!c.active) continue;
        se_cls_args a = make_cls_args(p, c, slot);
        int rows = p->D == 2 ? c.ny : p->g.Mg[1];
        int64_t n = 3 * (int64_t)c.nkx * rows * p->g.Mg[2];
        hipLaunchKernelGGL(k_cls_scatter<R>, dim3(nblk(n)), dim3(256), 0, s, a);
    }
}

template <typename R, int KER, int NC>
void cls_transform(const se_plan* p, int slot, hipStream_t s)
{
    for (const se_aft_class& c : p->cls) {
        if (!c.active) continue;
        se_fft_args f = cls_fft_args(p, c, slot);
        if (p->D == 1) run_y<R>(f, NC, 1, s);
        run_z_plain<R>(f, NC, 1, s);
        se_cls_args a = make_cls_args(p, c, slot);
        hipLaunchKernelGGL((k_cls_scale<R, KER, NC>), dim3(nblk((int64_t)c.nkx * c.ny * c.nz)), dim3(256), 0, s, a);
        run_z_plain<R>(f, 3, -1, s);
        if (p->D == 1) run_y<R>(f, 3, -1, s);
    }
}

template <typename R>
void cls_transform_dispatch(const se_plan* p, int slot, hipStream_t s)
{
    if (p->kernel == SE_STOKESLET) cls_transform<R, SE_STOKESLET, 3>(p, slot, s);
    else if (p->kernel == SE_ROTLET) cls_transform<R, SE_ROTLET, 3>(p, slot, s);
    else if (p->kernel == SE_HARMONIC) cls_transform<R, SE_HARMONIC, 3>(p, slot, s);
    else cls_transform<R, SE_STRESSLET, 6>(p, slot, s);
}

}  // namespace

// D = 1: the class planes are copied out after the x transform (before y);
// D = 2: the class columns after the x and y transforms.
namespace {

// ------------------------------------------------ direct k-space reference
// Triply periodic Fourier part as the explicit lattice sum (Sec. 2.2, eq.
// fourier-space-potential-3p) over the half space of k with 0 < |k| <= kmax:
//   S(k) = sum_n F_n e^{-i k.x_n},  U(k) = (2/V) Ghat^F(k) S(k),
//   u(x) += Re sum_k U(k) e^{i k.x}
// (the -k half is the complex conjugate).  F_n is f_n, or the symmetric
// part of q_n nu_n^T (6 components) for the stresslet; Ghat^F is the same
// scalar-times-operator form as the grid scaling, without the window.
struct se_dref_k_args {
    int nk;
    const double* kv;  // [nk][3]
    int64_t ns;
    const double* xs;  // [ns][3]
    const double* f;   // [ns][3]
    const double* nu;  // [ns][3] (stresslet)
    double xi, scale;  // scale = 2 / V
    double* U;         // [nk][3] complex (6 doubles per k)
    int64_t nt;
    const double* xt;  // [nt][3]
    double* u;         // [nt][3], accumulated
};

template <int KER, int NC>
__global__ void __launch_bounds__(256) k_dref_sk(se_dref_k_args a)
{
    __shared__ double red[NC * 2][256];
    const int ik = blockIdx.x, t = threadIdx.x;
    const double k[3] = {a.kv[3 * ik], a.kv[3 * ik + 1], a.kv[3 * ik + 2]};
    double sr[NC], si[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) sr[c] = si[c] = 0.0;
    for (int64_t n = t; n < a.ns; n += 256) {
        const double th = -(k[0] * a.xs[3 * n] + k[1] * a.xs[3 * n + 1] + k[2] * a.xs[3 * n + 2]);
        double sn, cs;
        sincos(th, &sn, &cs);
        double F[NC];
        if constexpr (NC == 3) {
#pragma unroll
            for (int c = 0; c < 3; c++) F[c] = a.f[3 * n + c];
        } else {
            const double q[3] = {a.f[3 * n], a.f[3 * n + 1], a.f[3 * n + 2]};
            const double v[3] = {a.nu[3 * n], a.nu[3 * n + 1], a.nu[3 * n + 2]};
            F[0] = q[0] * v[0];
            F[1] = q[1] * v[1];
            F[2] = q[2] * v[2];
            F[3] = 0.5 * (q[0] * v[1] + q[1] * v[0]);
            F[4] = 0.5 * (q[0] * v[2] + q[2] * v[0]);
            F[5] = 0.5 * (q[1] * v[2] + q[2] * v[1]);
        }
#pragma unroll
        for (int c = 0; c < NC; c++) {
            sr[c] += F[c] * cs;
            si[c] += F[c] * sn;
        }
    }
#pragma unroll
    for (int c = 0; c < NC; c++) {
        red[2 * c][t] = sr[c];
        red[2 * c + 1][t] = si[c];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int c = 0; c < 2 * NC; c++) red[c][t] += red[c][t + off];
        __syncthreads();
    }
    if (t == 0) {
        C<double> F[NC], U[3];
#pragma unroll
        for (int c = 0; c < NC; c++) F[c] = {red[2 * c][0], red[2 * c + 1][0]};
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double e = k2 / (4.0 * a.xi * a.xi);
        const double gE = exp(-e);
        const double screen = se_harmonic_based(KER) ? gE : gE * (1.0 + e);
        const double G = se_harmonic_based(KER) ? 4.0 * M_PI / k2 : -8.0 * M_PI / (k2 * k2);
        apply_green<double, KER>(G * screen * a.scale, k, k2, F, U);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            a.U[6 * ik + 2 * j] = U[j].x;
            a.U[6 * ik + 2 * j + 1] = U[j].y;
        }
    }
}

// one thread per target; the k list passes through LDS in tiles
__global__ void __launch_bounds__(256) k_dref_keval(se_dref_k_args a)
{
    __shared__ double sk[256][3];
    __shared__ double su[256][6];
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x[3] = {0.0, 0.0, 0.0};
    if (m < a.nt)
        for (int d = 0; d < 3; d++) x[d] = a.xt[3 * m + d];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int base = 0; base < a.nk; base += 256) {
        const int i = base + threadIdx.x;
        if (i < a.nk) {
            for (int d = 0; d < 3; d++) sk[threadIdx.x][d] = a.kv[3 * i + d];
            for (int d = 0; d < 6; d++) su[threadIdx.x][d] = a.U[6 * i + d];
        }
        __syncthreads();
        const int cnt = min(256, a.nk - base);
        for (int j = 0; j < cnt; j++) {
            const double th = sk[j][0] * x[0] + sk[j][1] * x[1] + sk[j][2] * x[2];
            double sn, cs;
            sincos(th, &sn, &cs);
#pragma unroll
            for (int c = 0; c < 3; c++) acc[c] += su[j][2 * c] * cs - su[j][2 * c + 1] * sn;
        }
        __syncthreads();
    }
    if (m < a.nt)
        for (int c = 0; c < 3; c++) a.u[3 * m + c] += acc[c];
}

}  // namespace

void se_launch_dref_kspace(int kernel, int nk, const double* kv, double xi, double volume, int64_t ns,
                           const double* xs, const double* f, const double* nu, double* U, int64_t nt,
                           const double* xt, double* u, hipStream_t s)
{
    se_dref_k_args a;
    a.nk = nk;
    a.kv = kv;
    a.ns = ns;
    a.xs = xs;
    a.f = f;
    a.nu = nu;
    a.xi = xi;
    a.scale = 2.0 / volume;
    a.U = U;
    a.nt = nt;
    a.xt = xt;
    a.u = u;
    if (nk > 0) {
        if (kernel == SE_STOKESLET) hipLaunchKernelGGL((k_dref_sk<SE_STOKESLET, 3>), dim3(nk), dim3(256), 0, s, a);
        else if (kernel == SE_ROTLET) hipLaunchKernelGGL((k_dref_sk<SE_ROTLET, 3>), dim3(nk), dim3(256), 0, s, a);
        else if (kernel == SE_HARMONIC) hipLaunchKernelGGL((k_dref_sk<SE_HARMONIC, 3>), dim3(nk), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_dref_sk<SE_STRESSLET, 6>), dim3(nk), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_dref_keval, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, a);
    }
}

void se_launch_fft_xy_forward(const se_plan* p, int slot, hipStream_t s)
{
    if (p->fp32) launch_fwd<float>(p, slot, s);
    else launch_fwd<double>(p, slot, s);
}

void se_launch_fft_z_scale(const se_plan* p, int slot, hipStream_t s)
{
    if (p->fp32) {
        launch_z_dispatch<float>(p, slot, s);
        if (p->D == 1 || p->D == 2) cls_transform_dispatch<float>(p, slot, s);
        if (p->D == 2) cls_scatter<float>(p, slot, s);
    } else {
        launch_z_dispatch<double>(p, slot, s);
        if (p->D == 1 || p->D == 2) cls_transform_dispatch<double>(p, slot, s);
        if (p->D == 2) cls_scatter<double>(p, slot, s);
    }
}

void se_launch_fft_inverse(const se_plan* p, int slot, hipStream_t s)
{
    if (p->fp32) launch_inv<float>(p, slot, s);
    else launch_inv<double>(p, slot, s);
}

// Whether the line kernels can hold the transforms of a plan in LDS
// (one column at least per bundle, 160 KB per workgroup).
// The dynamic LDS of a line kernel plus its static part (the radix table)
// must fit the 160 KiB a workgroup may hold: a dispatch asking for more is
// refused by the runtime and takes the queue down with it.
bool se_fft_fits(const int* N, int ncomp, bool fp32)
{
    const size_t cb = fp32 ? 8 : 16;
    const size_t lim = 160 * 1024 - kFftLdsStatic;
    const size_t nh = (size_t)N[0] / 2;
    return (2 * nh + 1 + 2 * nh) * cb <= lim && (size_t)N[1] * 3 * cb <= lim && (size_t)N[2] * 3 * cb <= lim &&
           (size_t)N[2] * (1 + (ncomp + 1)) * cb <= lim &&
           ((size_t)N[2] * (1 + ncomp) + (size_t)kZSetPad * ncomp) * cb <= lim;
}

// FP64 3-D transform of ncomp components on an arbitrary grid:
// dir > 0: real grid [c][Mg2][Mg1][Mg0] (zero padded to N) -> half spectrum
// [c][Mg2][N1][N0/2+1] with z transformed in place over N2 (requires Mg2 == N2);
// dir < 0: the reverse (C2R, truncated to Mg).  Unnormalised.
void se_fft3d_f64(const int* Mg, const int* N, const double* h, double* grid, double* spec, const double* tw,
                  const int* tw_off, int ncomp, int dir, hipStream_t s)
{
    se_fft_args a = make_fft_args_geom(Mg, N, h, grid, spec, tw, tw_off, ncomp);
    if (dir > 0) {
        run_x_r2c<double>(a, ncomp, s);
        run_y<double>(a, ncomp, 1, s);
        run_z_plain<double>(a, ncomp, 1, s);
    } else {
        run_z_plain<double>(a, ncomp, -1, s);
        run_y<double>(a, ncomp, -1, s);
        run_x_c2r<double>(a, ncomp, s);
    }
}

// ---------------------------------------------------------------------------
// Jobs of merged batches: the records, workgroups and LDS that the
// single-plan launchers above choose.  Variant: bit 0 FP32, bit 1 the
// long-line kernels; the fused z pass adds the kernel type (bits 2-4) and 6
// components (bit 5).
namespace {

template <typename R>
void fft_job(const se_plan* p, int family, int slot, std::vector<se_job>* out)
{
    se_job j;
    j.family = family;
    se_fft_args a;
    int Nline = 0;
    if (family == SE_JOB_FFT_X_R2C || family == SE_JOB_FFT_X_C2R) {
        const int nc = family == SE_JOB_FFT_X_R2C ? p->ncomp : 3;
        a = make_fft_args(p, nc, slot);
        const int Nh = a.N[0] / 2;
        a.ncomp = nc;
        a.lines = x_lines<R>(Nh);
        const int64_t rows = (int64_t)nc * a.Mg[2] * a.Mg[1];
        j.blocks = (int)((rows + a.lines - 1) / a.lines);
        j.lds = (size_t)(2 * Nh + 1 + a.lines * Nh) * sizeof(C<R>);
        Nline = Nh;
    } else if (family == SE_JOB_FFT_Y_FWD || family == SE_JOB_FFT_Y_INV) {
        const int nc = family == SE_JOB_FFT_Y_FWD ? p->ncomp : 3;
        a = make_fft_args(p, nc, slot);
        a.cols = bundle_cols<R>(a.N[1], 1, a.cols_cap);
        const int nbx = (a.Hx + a.cols - 1) / a.cols;
        j.blocks = nbx * nc * a.Mg[2];
        j.lds = (size_t)(a.N[1] + a.cols * a.N[1]) * sizeof(C<R>);
        Nline = a.N[1];
    } else {
        const int NC = p->kernel == SE_STRESSLET ? 6 : 3;
        a = make_fft_args(p, NC, slot);
        a.cols = bundle_cols<R>(p->Nfft[2], NC, p->shape_fft_cols > 0 ? p->shape_fft_cols : 2, kZSetPad);
        const int nbx = (p->Hx + a.cols - 1) / a.cols;
        j.blocks = nbx * p->Nfft[1];
        j.lds = (size_t)(p->Nfft[2] + NC * (a.cols * p->Nfft[2] + kZSetPad)) * sizeof(C<R>);
        Nline = p->Nfft[2];
        j.variant = (p->kernel << 2) | (NC == 6 ? 32 : 0);
    }
    j.variant |= (p->fp32 ? 1 : 0) | (Nline > kIpElems ? 2 : 0);
    j.args.resize(sizeof(se_fft_args));
    std::memcpy(j.args.data(), &a, sizeof(a));
    out->push_back(std::move(j));
}

template <typename K>
void multi_launch(K kern, const void* args, const int* boff, int n, int blocks, size_t lds, hipStream_t s)
{
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(SE_FFT_THREADS), lds, s, (const se_fft_args*)args, boff, n);
}

template <typename R, int E>
void fft_multi_e(int family, int variant, const void* args, const int* boff, int n, int blocks, size_t lds,
                 hipStream_t s)
{
    switch (family) {
        case SE_JOB_FFT_X_R2C: multi_launch(k_fft_x_r2c_multi<R, E>, args, boff, n, blocks, lds, s); break;
        case SE_JOB_FFT_X_C2R: multi_launch(k_fft_x_c2r_multi<R, E>, args, boff, n, blocks, lds, s); break;
        case SE_JOB_FFT_Y_FWD: multi_launch(k_fft_y_multi<R, E, 1>, args, boff, n, blocks, lds, s); break;
        case SE_JOB_FFT_Y_INV: multi_launch(k_fft_y_multi<R, E, -1>, args, boff, n, blocks, lds, s); break;
        default: {
            const int ker = (variant >> 2) & 7;
            if (ker == SE_STOKESLET)
                multi_launch(k_fft_z_scale_multi<R, SE_STOKESLET, 3, E>, args, boff, n, blocks, lds, s);
            else if (ker == SE_ROTLET)
                multi_launch(k_fft_z_scale_multi<R, SE_ROTLET, 3, E>, args, boff, n, blocks, lds, s);
            else if (ker == SE_HARMONIC)
                multi_launch(k_fft_z_scale_multi<R, SE_HARMONIC, 3, E>, args, boff, n, blocks, lds, s);
            else
                multi_launch(k_fft_z_scale_multi<R, SE_STRESSLET, 6, E>, args, boff, n, blocks, lds, s);
        }
    }
}

}  // namespace

bool se_fft_jobs(const se_plan* p, int family, int slot, std::vector<se_job>* out)
{
    if (p->fp32) fft_job<float>(p, family, slot, out);
    else fft_job<double>(p, family, slot, out);
    return true;
}

void se_fft_launch_multi(int family, int variant, const void* args, const int* boff, int n, int blocks, size_t lds,
                         hipStream_t s)
{
    if (n <= 0 || blocks <= 0) return;
    const bool fp32 = variant & 1, lng = variant & 2;
    if (fp32) {
        if (lng) fft_multi_e<float, kIpElemsLong>(family, variant, args, boff, n, blocks, lds, s);
        else fft_multi_e<float, kIpElems>(family, variant, args, boff, n, blocks, lds, s);
    } else {
        if (lng) fft_multi_e<double, kIpElemsLong>(family, variant, args, boff, n, blocks, lds, s);
        else fft_multi_e<double, kIpElems>(family, variant, args, boff, n, blocks, lds, s);
    }
}

void se_launch_fft_cls(const se_plan* p, int slot, int which, hipStream_t s)
{
    if (p->fp32) {
        if (which == 0 && p->D == 1) cls_gather<float>(p, slot, s);
        if (which == 1 && p->D == 2) cls_gather<float>(p, slot, s);
        if (which == 2 && (p->D == 1 || p->D == 2)) cls_transform_dispatch<float>(p, slot, s);
        if (which == 2 && p->D == 2) cls_scatter<float>(p, slot, s);
        if (which == 3 && p->D == 1) cls_scatter<float>(p, slot, s);
    } else {
        if (which == 0 && p->D == 1) cls_gather<double>(p, slot, s);
        if (which == 1 && p->D == 2) cls_gather<double>(p, slot, s);
        if (which == 2 && (p->D == 1 || p->D == 2)) cls_transform_dispatch<double>(p, slot, s);
        if (which == 2 && p->D == 2) cls_scatter<double>(p, slot, s);
        if (which == 3 && p->D == 1) cls_scatter<double>(p, slot, s);
    }
}
