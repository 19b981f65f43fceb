// se_real.hip -- real-space part (eq. real-space-potential-Dp) on the cell
// list, strength staging, FP64 reductions and the epilogue that adds the
// self term (eq. 3p-stokeslet-self-term), the non-periodic stresslet term
// (eq. k0-stresslet-3p) and scatters back to the caller's order.
#include "se_device.h"

namespace {

const double kSqrtPi = 1.7724538509055160272981675;

struct se_real_args {
    se_grid_geom g;
    const double* xt;  // sorted targets SoA [3][nt]
    int64_t nt;
    const double* xs;  // sorted sources SoA [3][ns]
    int64_t ns;
    const double* f;   // sorted strengths FP64 SoA [3][ns] (f, or q for T)
    const double* nrm; // sorted normals SoA [3][ns] (T)
    const int* start;  // source cell starts
    double xi, rc2;
    int Ra[3];         // anchor reach ceil(rc/h)+1
    int tas;
    double* u;         // [3][nt]
    int* flags;
};

// u_j += G^R_{jl(m)}(r; xi) . f, eqs. (stokeslet-real), (rotlet-real), (stresslet-real)
template <int KER>
__device__ __forceinline__ void real_kernel(double xi, const double* r, double r2, const double* f,
                                            const double* nu, double* u)
{
    const double rn = sqrt(r2);
    const double ec = erfc(xi * rn);
    const double ga = exp(-xi * xi * r2) * (2.0 * xi / kSqrtPi);  // 2 xi e^{-xi^2 r^2}/sqrt(pi)
    if constexpr (KER == SE_STOKESLET) {
        const double c1 = ec / rn + ga;
        const double c2 = 2.0 * ga;
        const double rf = (r[0] * f[0] + r[1] * f[1] + r[2] * f[2]) / r2;
#pragma unroll
        for (int j = 0; j < 3; j++) u[j] += c1 * (f[j] + r[j] * rf) - c2 * f[j];
    } else if constexpr (KER == SE_ROTLET) {
        const double c1 = (ec / rn + ga) / r2;
        u[0] += c1 * (f[1] * r[2] - f[2] * r[1]);
        u[1] += c1 * (f[2] * r[0] - f[0] * r[2]);
        u[2] += c1 * (f[0] * r[1] - f[1] * r[0]);
    } else {
        const double c1 = 3.0 * ec / rn + (3.0 + 2.0 * xi * xi * r2) * ga;
        const double c2 = 2.0 * xi * xi * ga;  // 4 xi^3 e^{-xi^2 r^2}/sqrt(pi)
        const double rq = r[0] * f[0] + r[1] * f[1] + r[2] * f[2];
        const double rv = r[0] * nu[0] + r[1] * nu[1] + r[2] * nu[2];
        const double qv = f[0] * nu[0] + f[1] * nu[1] + f[2] * nu[2];
        const double a = -2.0 * rq * rv / (r2 * r2) * c1;
#pragma unroll
        for (int j = 0; j < 3; j++) u[j] += a * r[j] + c2 * (f[j] * rv + nu[j] * rq + r[j] * qv);
    }
}

template <int KER>
__global__ void __launch_bounds__(256) k_real(se_real_args a)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nt) return;
    const se_grid_geom& g = a.g;
    double xt[3] = {a.xt[t], a.xt[a.nt + t], a.xt[2 * a.nt + t]};
    int blo[3], bhi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int an = se_anchor(g, d, xt[d]);
        blo[d] = se_floordiv(an - a.Ra[d], g.B[d]);
        bhi[d] = se_floordiv(an + a.Ra[d], g.B[d]);
        if (!g.periodic[d]) {
            blo[d] = max(blo[d], 0);
            bhi[d] = min(bhi[d], g.nb[d] - 1);
        }
    }
    double acc[3] = {0.0, 0.0, 0.0};
    int coinc = 0;
    for (int bz = blo[2]; bz <= bhi[2]; bz++) {
        int kz = g.periodic[2] ? se_floordiv(bz, g.nb[2]) : 0;
        int wz = bz - kz * g.nb[2];
        double sz = kz * g.L[2];
        for (int by = blo[1]; by <= bhi[1]; by++) {
            int ky = g.periodic[1] ? se_floordiv(by, g.nb[1]) : 0;
            int wy = by - ky * g.nb[1];
            double sy = ky * g.L[1];
            for (int bx = blo[0]; bx <= bhi[0]; bx++) {
                int kx = g.periodic[0] ? se_floordiv(bx, g.nb[0]) : 0;
                int wx = bx - kx * g.nb[0];
                double sx = kx * g.L[0];
                int bin = (wz * g.nb[1] + wy) * g.nb[0] + wx;
                int s0 = a.start[bin], s1 = a.start[bin + 1];
                bool zero_shift = (kx == 0 && ky == 0 && kz == 0);
                for (int s = s0; s < s1; s++) {
                    double r[3] = {xt[0] - (a.xs[s] + sx), xt[1] - (a.xs[a.ns + s] + sy),
                                   xt[2] - (a.xs[2 * a.ns + s] + sz)};
                    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    if (r2 >= a.rc2) continue;
                    if (zero_shift && a.tas && s == t) continue;
                    if (r2 == 0.0) {
                        coinc = 1;
                        continue;
                    }
                    double f[3] = {a.f[s], a.f[a.ns + s], a.f[2 * a.ns + s]};
                    double nu[3] = {0.0, 0.0, 0.0};
                    if (KER == SE_STRESSLET) {
                        nu[0] = a.nrm[s];
                        nu[1] = a.nrm[a.ns + s];
                        nu[2] = a.nrm[2 * a.ns + s];
                    }
                    real_kernel<KER>(a.xi, r, r2, f, nu, acc);
                }
            }
        }
    }
    if (coinc) atomicOr(a.flags, SE_FLAG_COINCIDENT);
    a.u[t] = acc[0];
    a.u[a.nt + t] = acc[1];
    a.u[2 * a.nt + t] = acc[2];
}

// Sorted strengths: FP64 copy [3][ns] of f (or q) for the real-space sum and
// self term, the gridded components in grid precision [ncomp][ns]
// (f, or the symmetric part of q nu^T: xx, yy, zz, xy, xz, yz), and q.nu.
template <typename R>
__global__ void k_strengths(const double* __restrict__ f, const int* __restrict__ perm, int64_t n,
                            const double* __restrict__ nrm, int ncomp, double* __restrict__ f64,
                            R* __restrict__ fs, double* __restrict__ qn, int* flags)
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

// Deterministic single-workgroup reductions for the stresslet zero-mode term:
// out[0] = sum_n q_n.nu_n, out[1..3] = sum_n x_n (q_n.nu_n).
__global__ void __launch_bounds__(1024) k_reduce_qn(const double* __restrict__ qn, const double* __restrict__ xs,
                                                    int64_t n, double* out)
{
    __shared__ double sm[4][1024];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        double q = qn[i];
        a0 += q;
        a1 += xs[i] * q;
        a2 += xs[n + i] * q;
        a3 += xs[2 * n + i] * q;
    }
    sm[0][threadIdx.x] = a0;
    sm[1][threadIdx.x] = a1;
    sm[2][threadIdx.x] = a2;
    sm[3][threadIdx.x] = a3;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; c++) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sm[threadIdx.x][0];
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
    double* u;            // [nt][3] caller order (or null)
    double* u_real;
    double* u_four;
};

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
        if (a.u) a.u[3 * o + j] = ur + uf;
        if (a.u_real) a.u_real[3 * o + j] = ur;
        if (a.u_four) a.u_four[3 * o + j] = uf;
    }
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void se_launch_strengths(const se_plan* p, const double* f, hipStream_t s)
{
    if (p->fp32)
        hipLaunchKernelGGL(k_strengths<float>, dim3(grid1d(p->ns, 256)), dim3(256), 0, s, f, p->d_src_perm, p->ns,
                           p->d_nrm, p->ncomp, p->d_fs64, (float*)p->d_fs, p->d_fs64 + 3 * p->ns, p->d_flags);
    else
        hipLaunchKernelGGL(k_strengths<double>, dim3(grid1d(p->ns, 256)), dim3(256), 0, s, f, p->d_src_perm, p->ns,
                           p->d_nrm, p->ncomp, p->d_fs64, (double*)p->d_fs, p->d_fs64 + 3 * p->ns, p->d_flags);
}

void se_launch_reductions(const se_plan* p, hipStream_t s)
{
    if (p->kernel == SE_STRESSLET && p->D == 3)
        hipLaunchKernelGGL(k_reduce_qn, dim3(1), dim3(1024), 0, s, p->d_fs64 + 3 * p->ns, p->d_src, p->ns, p->d_red);
}

void se_launch_real_space(const se_plan* p, hipStream_t s)
{
    se_real_args a;
    a.g = p->g;
    a.xt = p->tas ? p->d_src : p->d_tgt;
    a.nt = p->nt;
    a.xs = p->d_src;
    a.ns = p->ns;
    a.f = p->d_fs64;
    a.nrm = p->d_nrm;
    a.start = p->d_src_start;
    a.xi = p->par.xi;
    a.rc2 = p->par.rc * p->par.rc;
    for (int d = 0; d < 3; d++) a.Ra[d] = (int)std::ceil(p->par.rc / p->g.h[d]) + 1;
    a.tas = p->tas ? 1 : 0;
    a.u = p->d_uR;
    a.flags = p->d_flags;
    unsigned nb = grid1d(p->nt, 256);
    if (p->kernel == SE_STOKESLET) hipLaunchKernelGGL(k_real<SE_STOKESLET>, dim3(nb), dim3(256), 0, s, a);
    else if (p->kernel == SE_ROTLET) hipLaunchKernelGGL(k_real<SE_ROTLET>, dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_real<SE_STRESSLET>, dim3(nb), dim3(256), 0, s, a);
}

void se_launch_finalize(const se_plan* p, const double* f, double* u, double* u_real, double* u_fourier,
                        hipStream_t s)
{
    (void)f;
    se_fin_args a;
    a.nt = p->nt;
    a.perm = p->tas ? p->d_src_perm : p->d_tgt_perm;
    a.uF = p->d_uF;
    a.uR = p->d_uR;
    a.f64 = p->d_fs64;
    a.xt = p->tas ? p->d_src : p->d_tgt;
    a.red = p->d_red;
    a.self_c = (p->kernel == SE_STOKESLET && p->tas) ? -4.0 * p->par.xi / kSqrtPi : 0.0;
    a.k0_c = (p->kernel == SE_STRESSLET && p->D == 3) ? -8.0 * M_PI / (p->g.L[0] * p->g.L[1] * p->g.L[2]) : 0.0;
    a.u = u;
    a.u_real = u_real;
    a.u_four = u_fourier;
    hipLaunchKernelGGL(k_finalize, dim3(grid1d(p->nt, 256)), dim3(256), 0, s, a);
}
