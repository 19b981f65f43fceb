// se_bie.hip -- boundary-integral driver: restarted GMRES over the plan's
// periodic stresslet sum, many right-hand sides in lock step.
//
// Discretised double-layer operator on surface nodes x_n (weights w_n, unit
// outward normals nu_n), with the singularity subtracted through the
// stresslet identity (Sec. 2.4, eq. stresslet-identity: the integral of
// T q0 nu over a closed surface is 4 pi q0 on the surface):
//   (D q)_m = sum_{n != m} w_n T^{DP}(x_m - x_n) (q_n - q_m) nu_n + 4 pi q_m
//           = SE[w q]_m - M_m q_m + 4 pi q_m,
//   M_m[j][l] = sum_{n != m} w_n T^{DP}_{jlk}(x_m - x_n) nu_{n,k},
// and the equations alpha q + D q = g (with outward normals alpha = +4 pi
// and -4 pi give the interior and exterior limits of the double layer).
#include <algorithm>
#include <cmath>
#include <vector>

#include "se_internal.h"

namespace {

// s[r][n][c] = w[n] v[r][n][c]
__global__ void k_bie_weight(int64_t n3, int64_t nr, const double* __restrict__ w, const double* __restrict__ v,
                             double* __restrict__ s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3 * nr) return;
    s[i] = w[(i % n3) / 3] * v[i];
}

// s[r][n][c] = w[n] (c == l0 + r), r < nr (zero for l0 + r > 2)
__global__ void k_bie_unit(int64_t n, int64_t nr, int l0, const double* __restrict__ w, double* __restrict__ s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n * nr) return;
    const int64_t r = i / (3 * n), m = (i / 3) % n;
    const int c = (int)(i % 3);
    s[i] = (c == l0 + r) ? w[m] : 0.0;
}

// M[l][m][j] = u[r][m][j] for the set r = l - l0 (columns of M)
__global__ void k_bie_take(int64_t n, int64_t nr, int l0, const double* __restrict__ u, double* __restrict__ M)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n * nr) return;
    const int64_t r = i / (3 * n);
    if (l0 + r > 2) return;
    M[(l0 + r) * 3 * n + (i - r * 3 * n)] = u[i];
}

// out[r][m][j] = u[r][m][j] - sum_l M[l][m][j] v[r][m][l] + c v[r][m][j]
__global__ void k_bie_apply(int64_t n, int64_t nr, double c, const double* __restrict__ M, const double* __restrict__ v,
                            const double* __restrict__ u, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nr) return;
    const int64_t m = i % n;
    const double* vm = v + 3 * i;
    for (int j = 0; j < 3; j++) {
        double acc = u[3 * i + j] + c * vm[j];
        for (int l = 0; l < 3; l++) acc -= M[l * 3 * n + 3 * m + j] * vm[l];
        out[3 * i + j] = acc;
    }
}

// h[i][r] = <V_i[r], x[r]> for i < nv: one workgroup per (i, r), fixed order
__global__ void __launch_bounds__(256) k_bie_dots(int64_t len, int64_t nr, const double* __restrict__ V,
                                                  int64_t vstride, const double* __restrict__ x, double* __restrict__ h)
{
    __shared__ double red[256];
    const int64_t i = blockIdx.x / nr, r = blockIdx.x % nr;
    const double* a = V + i * vstride + r * len;
    const double* b = x + r * len;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < len; k += 256) s += a[k] * b[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[i * nr + r] = red[0];
}

// x[r] += sgn sum_{i < nv} h[i][r] V_i[r]
__global__ void k_bie_combine(int64_t len, int64_t nr, int nv, const double* __restrict__ V, int64_t vstride,
                              const double* __restrict__ h, double sgn, double* __restrict__ x)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len * nr) return;
    const int64_t r = k / len;
    double acc = 0.0;
    for (int i = 0; i < nv; i++) acc += h[i * nr + r] * V[i * vstride + k];
    x[k] += sgn * acc;
}

// x = g - x
__global__ void k_bie_rsub(int64_t len, const double* __restrict__ g, double* __restrict__ x)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    x[k] = g[k] - x[k];
}

// y[r] = a[r] x[r]  (a on the device, one factor per system)
__global__ void k_bie_scale(int64_t len, int64_t nr, const double* __restrict__ a, const double* __restrict__ x,
                            double* __restrict__ y)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len * nr) return;
    y[k] = a[k / len] * x[k];
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Bie {
    se_plan* p;
    hipStream_t s;
    int64_t n, n3, R, vs;  // vs: length of one block of R vectors
    double c;              // alpha + 4 pi
    const double* w;
    double *M = nullptr, *S = nullptr, *U = nullptr, *hd = nullptr;
    hipError_t err = hipSuccess;

    bool ok(hipError_t e)
    {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return err == hipSuccess;
    }
    // out = (alpha I + D) v for all R systems
    se_status apply(const double* v, double* out)
    {
        hipLaunchKernelGGL(k_bie_weight, dim3(blocks_of(vs)), dim3(256), 0, s, n3, R, w, v, S);
        se_status st = se_run_plan(p, S, U, nullptr, nullptr, s);
        if (st != SE_OK) return st;
        hipLaunchKernelGGL(k_bie_apply, dim3(blocks_of(n * R)), dim3(256), 0, s, n, R, c, M, v, U, out);
        return ok(hipGetLastError()) ? SE_OK : SE_ERR_HIP;
    }
    // M from three evaluations with the unit densities q0 = e_l
    se_status build_m()
    {
        for (int l0 = 0; l0 < 3; l0 += (int)R) {
            hipLaunchKernelGGL(k_bie_unit, dim3(blocks_of(vs)), dim3(256), 0, s, n, R, l0, w, S);
            se_status st = se_run_plan(p, S, U, nullptr, nullptr, s);
            if (st != SE_OK) return st;
            hipLaunchKernelGGL(k_bie_take, dim3(blocks_of(vs)), dim3(256), 0, s, n, R, l0, U, M);
        }
        return ok(hipGetLastError()) ? SE_OK : SE_ERR_HIP;
    }
    // h[i][r] = <V_i[r], x[r]>, i < nv (V_i at stride vs), to the host
    bool dots(const double* V, int nv, const double* x, std::vector<double>& h)
    {
        hipLaunchKernelGGL(k_bie_dots, dim3((unsigned)(nv * R)), dim3(256), 0, s, n3, R, V, vs, x, hd);
        h.assign((size_t)nv * R, 0.0);
        return ok(hipGetLastError()) &&
               ok(hipMemcpyAsync(h.data(), hd, h.size() * sizeof(double), hipMemcpyDeviceToHost, s)) &&
               ok(hipStreamSynchronize(s));
    }
    // x[r] += sgn sum_i h[i][r] V_i[r]
    bool combine(const double* V, int nv, const std::vector<double>& h, double sgn, double* x)
    {
        if (!ok(hipMemcpyAsync(hd, h.data(), (size_t)nv * R * sizeof(double), hipMemcpyHostToDevice, s))) return false;
        hipLaunchKernelGGL(k_bie_combine, dim3(blocks_of(vs)), dim3(256), 0, s, n3, R, nv, V, vs, hd, sgn, x);
        return ok(hipGetLastError()) && ok(hipStreamSynchronize(s));
    }
    // y[r] = a[r] x[r]
    bool scale(const std::vector<double>& a, const double* x, double* y)
    {
        if (!ok(hipMemcpyAsync(hd, a.data(), R * sizeof(double), hipMemcpyHostToDevice, s))) return false;
        hipLaunchKernelGGL(k_bie_scale, dim3(blocks_of(vs)), dim3(256), 0, s, n3, R, hd, x, y);
        return ok(hipGetLastError()) && ok(hipStreamSynchronize(s));
    }
};

}  // namespace

extern "C" se_status se_bie_solve(se_plan* plan, double alpha, const double* weights, const double* g, double* q,
                                  int32_t restart, int32_t max_iter, double tol, int32_t* iters, double* resid,
                                  void* stream)
{
    if (!plan || !weights || !g || !q || restart < 1 || restart > 200 || max_iter < 1 || !(tol > 0) ||
        !std::isfinite(alpha))
        return SE_ERR_ARG;
    if (plan->kernel != SE_STRESSLET || !plan->tas) return SE_ERR_ARG;
    if (!plan->have_geometry) return SE_ERR_STATE;
    if (hipSetDevice(plan->device) != hipSuccess) return SE_ERR_HIP;
    Bie B;
    B.p = plan;
    B.s = (hipStream_t)stream;
    B.n = plan->ns;
    B.n3 = 3 * plan->ns;
    B.R = plan->nrhs;
    B.vs = B.n3 * B.R;
    B.c = alpha + 4.0 * M_PI;
    B.w = weights;
    const int64_t R = B.R, vs = B.vs;
    const int J = restart;
    double *V = nullptr, *Wv = nullptr;
    se_status st = SE_OK;
    auto alloc = [&](double** p, size_t cnt) {
        if (st == SE_OK && !B.ok(hipMalloc(p, cnt * sizeof(double))))
            st = B.err == hipErrorOutOfMemory ? SE_ERR_NOMEM : SE_ERR_HIP;
        return st == SE_OK;
    };
    std::vector<double> bnorm(R, 0.0), res(R, 0.0);
    int used = 0;
    alloc(&B.M, 3 * (size_t)B.n3);
    alloc(&B.S, (size_t)vs);
    alloc(&B.U, (size_t)vs);
    alloc(&V, (size_t)(J + 1) * vs);
    alloc(&Wv, (size_t)vs);
    alloc(&B.hd, (size_t)(J + 1) * R);
    std::vector<double> h, h2;
    if (st == SE_OK) st = B.build_m();
    if (st == SE_OK) {
        if (B.dots(g, 1, g, h))
            for (int r = 0; r < R; r++) bnorm[r] = std::sqrt(h[r]);
        else
            st = SE_ERR_HIP;
    }
    while (st == SE_OK) {
        // true residual r = g - A q and its relative norm
        st = B.apply(q, Wv);
        if (st != SE_OK) break;
        hipLaunchKernelGGL(k_bie_rsub, dim3(blocks_of(vs)), dim3(256), 0, B.s, vs, g, Wv);
        if (!B.dots(Wv, 1, Wv, h)) {
            st = SE_ERR_HIP;
            break;
        }
        std::vector<double> beta(R), inv(R);
        bool all = true;
        for (int r = 0; r < R; r++) {
            beta[r] = std::sqrt(h[r]);
            res[r] = bnorm[r] > 0 ? beta[r] / bnorm[r] : beta[r];
            all = all && res[r] <= tol;
            inv[r] = beta[r] > 1e-300 ? 1.0 / beta[r] : 0.0;
        }
        if (all || used >= max_iter) break;
        if (!B.scale(inv, Wv, V)) {
            st = SE_ERR_HIP;
            break;
        }
        // one cycle: Arnoldi (classical Gram-Schmidt twice), Givens per system
        std::vector<double> H((size_t)(J + 1) * J * R, 0.0), cs((size_t)J * R, 1.0), sn((size_t)J * R, 0.0),
            e((size_t)(J + 1) * R, 0.0);
        auto Hat = [&](int i, int j, int r) -> double& { return H[((size_t)i * J + j) * R + r]; };
        for (int r = 0; r < R; r++) e[r] = beta[r];
        int k = 0;
        while (k < J && used < max_iter) {
            const int j = k;
            st = B.apply(V + (size_t)j * vs, Wv);
            if (st != SE_OK) break;
            used++;
            if (!B.dots(V, j + 1, Wv, h) || !B.combine(V, j + 1, h, -1.0, Wv) || !B.dots(V, j + 1, Wv, h2) ||
                !B.combine(V, j + 1, h2, -1.0, Wv)) {
                st = SE_ERR_HIP;
                break;
            }
            for (size_t t = 0; t < h.size(); t++) h[t] += h2[t];
            std::vector<double> nn;
            if (!B.dots(Wv, 1, Wv, nn)) {
                st = SE_ERR_HIP;
                break;
            }
            std::vector<double> ihn(R);
            bool conv = true;
            for (int r = 0; r < R; r++) {
                const double hn = std::sqrt(nn[r]);
                ihn[r] = hn > 1e-300 ? 1.0 / hn : 0.0;
                for (int i = 0; i <= j; i++) Hat(i, j, r) = h[(size_t)i * R + r];
                Hat(j + 1, j, r) = hn;
                for (int i = 0; i < j; i++) {
                    const double a = Hat(i, j, r), b = Hat(i + 1, j, r);
                    Hat(i, j, r) = cs[i * R + r] * a + sn[i * R + r] * b;
                    Hat(i + 1, j, r) = -sn[i * R + r] * a + cs[i * R + r] * b;
                }
                const double a = Hat(j, j, r), b = Hat(j + 1, j, r), rr = std::hypot(a, b);
                cs[j * R + r] = rr > 0 ? a / rr : 1.0;
                sn[j * R + r] = rr > 0 ? b / rr : 0.0;
                Hat(j, j, r) = rr;
                Hat(j + 1, j, r) = 0.0;
                e[(size_t)(j + 1) * R + r] = -sn[j * R + r] * e[(size_t)j * R + r];
                e[(size_t)j * R + r] = cs[j * R + r] * e[(size_t)j * R + r];
                const double est = std::fabs(e[(size_t)(j + 1) * R + r]);
                res[r] = bnorm[r] > 0 ? est / bnorm[r] : est;
                conv = conv && res[r] <= tol;
            }
            if (!B.scale(ihn, Wv, V + (size_t)(j + 1) * vs)) {
                st = SE_ERR_HIP;
                break;
            }
            k = j + 1;
            if (conv) break;
        }
        if (st != SE_OK || k == 0) break;
        // y = H^{-1} e (upper triangular k x k), q += V y
        std::vector<double> y((size_t)k * R, 0.0);
        for (int r = 0; r < R; r++)
            for (int i = k - 1; i >= 0; i--) {
                double acc = e[(size_t)i * R + r];
                for (int t = i + 1; t < k; t++) acc -= Hat(i, t, r) * y[(size_t)t * R + r];
                const double d = Hat(i, i, r);
                y[(size_t)i * R + r] = std::fabs(d) > 1e-300 ? acc / d : 0.0;
            }
        if (!B.combine(V, k, y, 1.0, q)) st = SE_ERR_HIP;
    }
    if (iters) *iters = used;
    if (resid)
        for (int r = 0; r < R; r++) resid[r] = res[r];
    hipStreamSynchronize(B.s);
    for (double* p : {B.M, B.S, B.U, V, Wv, B.hd})
        if (p) hipFree(p);
    return st;
}
