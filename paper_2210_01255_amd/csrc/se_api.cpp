// se_api.cpp -- the C ABI: plan lifecycle, geometry binding and execution.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <thread>

#include "se_internal.h"

// defined in se_spread.hip
void se_tile_shape(int ncomp, bool fp32, int* tile);

namespace {

struct Alloc {
    se_plan* p;
    bool ok = true;
    template <typename T>
    T* get(size_t count)
    {
        if (!ok || count == 0) return nullptr;
        void* ptr = nullptr;
        size_t bytes = count * sizeof(T);
        bytes = (bytes + 255) & ~(size_t)255;
        if (hipMalloc(&ptr, bytes) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        p->ws_bytes += bytes;
        return (T*)ptr;
    }
};

void free_all(se_plan* p)
{
    void* ptrs[] = {p->d_flags, p->d_src, p->d_nrm, p->d_src_perm, p->d_src_start, p->d_tgt, p->d_tgt_perm,
                    p->d_tgt_start, p->d_keys_a, p->d_keys_b, p->d_vals_a, p->d_sort_tmp, p->d_fs, p->d_fs64,
                    p->d_red, p->d_grid, p->d_spec, p->d_uF, p->d_uR, p->d_pkb, p->d_invw2, p->d_tw,
                    p->d_pos4, p->d_tpos4, p->d_str4, p->d_nrm4, p->d_rtab, p->d_ktab, p->d_rwork,
                    p->d_rtx_s, p->d_rtx_t};
    for (void* q : ptrs)
        if (q) hipFree(q);
    for (se_aft_class& c : p->cls) {
        void* cp[] = {c.buf, c.kv, c.iw, c.tw, c.mk};
        for (void* q : cp)
            if (q) hipFree(q);
    }
}

// Class shapes of the adaptive transform (Sec. 3.4): [0] k^P = 0 with the
// upsampled lengths s0 M'_i, [1] the set K_* (|k_i| <= k*, k^P != 0) with
// s_* M'_i.  The threshold is clipped below the Nyquist index of each
// periodic axis.
void aft_shapes(se_plan* p)
{
    const se_params& par = p->par;
    for (se_aft_class& c : p->cls) c = se_aft_class();
    if (p->D != 1 && p->D != 2) return;
    const int kx = std::max(0, std::min(par.kstar[0], p->Nfft[0] / 2 - 1));
    const int ky = p->D == 2 ? std::max(0, std::min(par.kstar[1], p->Nfft[1] / 2 - 1)) : 0;
    se_aft_class& c0 = p->cls[0];
    c0.active = 1;
    c0.zero = 1;
    c0.nkx = 1;
    c0.kx_lo = 0;
    c0.ky_lo = 0;
    se_aft_class& c1 = p->cls[1];
    c1.active = p->D == 2 ? (kx >= 1 || ky >= 1) : kx >= 1;
    if (p->D == 2) {
        c0.ny = 1;
        c0.nz = par.n0_fft[2];
        c1.nkx = kx + 1;
        c1.ny = 2 * ky + 1;
        c1.nz = par.nstar_fft[2];
        c1.kx_lo = 0;
        c1.ky_lo = -ky;
    } else {
        c0.ny = par.n0_fft[1];
        c0.nz = par.n0_fft[2];
        c1.nkx = kx;
        c1.ny = par.nstar_fft[1];
        c1.nz = par.nstar_fft[2];
        c1.kx_lo = 1;
        c1.ky_lo = 0;
    }
    if (!c1.active) c1.nkx = c1.ny = c1.nz = 0;
}

// 1 - J0(x) and 1 - J0(x) - x J1(x)/2 (series for small x)
void bessel_brackets(double x, double* h, double* b)
{
    if (x < 0.5) {
        long double q = (long double)x * x / 4.0L, t = 1.0L, sh = 0.0L, sb = 0.0L;
        for (int m = 1; m < 30; m++) {
            t *= -q / ((long double)m * m);  // (-1)^m (x/2)^{2m} / (m!)^2
            sh -= t;
            sb += t * (m - 1);
        }
        *h = (double)sh;
        *b = (double)sb;
        return;
    }
    const double j0 = std::cyl_bessel_j(0.0, x), j1 = std::cyl_bessel_j(1.0, x);
    *h = 1.0 - j0;
    *b = 1.0 - j0 - 0.5 * x * j1;
}

// Wavenumbers, window deconvolution, twiddles and (D = 1, k^P = 0) the
// modified kernels Hhat_R^{1P}, Bhat_R^{1P} (eqs. optimal-1p-harmonic,
// optimal-1p-biharmonic with their limits) of each active class.
hipError_t aft_tables(se_plan* p)
{
    const se_params& par = p->par;
    const double twopi = 2.0 * M_PI;
    for (se_aft_class& c : p->cls) {
        if (!c.active) continue;
        std::vector<double> kv, iw;
        const int n[3] = {c.nkx, c.ny, c.nz};
        double nv[3];
        for (int d = 0; d < 3; d++) {
            const double a = par.h[d] * par.P / 2.0;
            const bool periodic = d < p->D;
            for (int i = 0; i < n[d]; i++) {
                double k;
                if (d == 0) k = twopi * (c.kx_lo + i) / p->g.L[0];
                else if (periodic) k = twopi * (c.ky_lo + i) / p->g.L[1];
                else k = twopi * (i < n[d] / 2 ? i : i - n[d]) / (par.h[d] * n[d]);
                kv.push_back(k);
                double w = se_window_fourier(par, k, a);
                iw.push_back(1.0 / (w * w));
            }
            nv[d] = periodic ? p->Nfft[d] : n[d];
        }
        c.scale = par.h[0] * par.h[1] * par.h[2] / (nv[0] * nv[1] * nv[2]);
        std::vector<double> tw;
        const int Nt[3] = {2, c.ny, c.nz};
        se_fft_twiddles(Nt, &tw, c.tw_off);
        hipError_t e = hipMemcpy(c.kv, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c.iw, iw.data(), iw.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c.tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        if (c.mk) {
            // the multipliers depend on |k| only and the free-axis wavenumbers
            // of index i and n - i are opposite: evaluate one quadrant (the
            // Bessel functions dominate plan creation) on host threads, then
            // mirror it
            const double R = par.R;
            const int qy = c.ny / 2 + 1, qz = c.nz / 2 + 1;
            std::vector<double> quad((size_t)2 * qy * qz);
            auto rows = [&](int z0, int z1) {
                for (int iz = z0; iz < z1; iz++)
                    for (int iy = 0; iy < qy; iy++) {
                        const double ky = kv[c.nkx + iy], kz = kv[c.nkx + c.ny + iz];
                        const double kk = std::sqrt(ky * ky + kz * kz);
                        double hb, bb;
                        bessel_brackets(R * kk, &hb, &bb);
                        double H, B;
                        if (kk == 0.0) {
                            H = M_PI * R * R;
                            B = -M_PI * R * R * R * R / 8.0;
                        } else {
                            H = 4.0 * M_PI / (kk * kk) * hb;
                            B = -8.0 * M_PI / (kk * kk * kk * kk) * bb;
                        }
                        quad[2 * ((size_t)iz * qy + iy)] = H;
                        quad[2 * ((size_t)iz * qy + iy) + 1] = B;
                    }
            };
            const int nth = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
            std::vector<std::thread> pool;
            for (int t = 0; t < nth; t++) pool.emplace_back(rows, (int)((int64_t)qz * t / nth),
                                                            (int)((int64_t)qz * (t + 1) / nth));
            for (auto& th : pool) th.join();
            std::vector<double> mk((size_t)2 * c.ny * c.nz);
            for (int iz = 0; iz < c.nz; iz++) {
                const int jz = std::min(iz, c.nz - iz);
                for (int iy = 0; iy < c.ny; iy++) {
                    const int jy = std::min(iy, c.ny - iy);
                    mk[2 * ((size_t)iz * c.ny + iy)] = quad[2 * ((size_t)jz * qy + jy)];
                    mk[2 * ((size_t)iz * c.ny + iy) + 1] = quad[2 * ((size_t)jz * qy + jy) + 1];
                }
            }
            e = hipMemcpy(c.mk, mk.data(), mk.size() * sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int key_bits(int64_t nbins)
{
    int b = 1;
    while ((int64_t(1) << b) <= nbins) b++;
    return b;
}

se_status check_hip(se_plan* p, hipError_t e, const char* what)
{
    if (e == hipSuccess) return SE_OK;
    if (p) p->msg = std::string(what) + ": " + hipGetErrorString(e);
    return SE_ERR_HIP;
}

}  // namespace

// Twiddle tables (complex FP64, interleaved) for the R2C axis (the stages of
// length N0/2, and the split factors e^{-2 pi i k/N0} for k = 0..N0/2) and
// the y and z axes.  A line length n has n entries: for each Stockham stage
// (in the order of se_fft_radix_order) with Ns = the product of the earlier
// radices, the factors e^{-2 pi i r jn/(Ns RAD)}, r = 1..RAD-1 major and
// jn = 0..Ns-1 minor, from entry Ns - 1 (the stages fill n - 1 entries).
void se_fft_twiddles(const int* N, std::vector<double>* tw, int* off)
{
    tw->clear();
    const int Nh = N[0] / 2;
    const long double twopi = 2.0L * 3.141592653589793238462643383279502884L;
    auto push = [&](long double ang) {
        tw->push_back((double)std::cos(ang));
        tw->push_back((double)std::sin(ang));
    };
    // exactly n entries per table (the offsets below assume it); a length
    // that is not 7-smooth (a class axis no line transform runs along) gets
    // unit entries
    auto push_stages = [&](int n) {
        const size_t end = tw->size() + 2 * (size_t)n;
        std::vector<int> rad;
        if (se_fft_radix_order(n, &rad)) {
            int Ns = 1;
            for (int R : rad) {
                for (int r = 1; r < R; r++)
                    for (int jn = 0; jn < Ns; jn++) push(-twopi * r * jn / ((long double)Ns * R));
                Ns *= R;
            }
        }
        while (tw->size() < end) push(0.0L);
    };
    off[0] = 0;
    push_stages(Nh);
    off[1] = Nh;
    for (int k = 0; k <= Nh; k++) push(-twopi * k / N[0]);
    off[2] = 2 * Nh + 1;
    push_stages(N[1]);
    off[3] = 2 * Nh + 1 + N[1];
    push_stages(N[2]);
}

extern "C" {

int32_t se_version(void) { return SE_VERSION_MAJOR * 10000 + SE_VERSION_MINOR * 100 + SE_VERSION_PATCH; }

const char* se_status_string(se_status s)
{
    switch (s) {
        case SE_OK: return "ok";
        case SE_ERR_ARG: return "invalid argument";
        case SE_ERR_UNSUPPORTED: return "unsupported request";
        case SE_ERR_OUT_OF_BOX: return "point outside the primary cell";
        case SE_ERR_NONFINITE: return "non-finite input";
        case SE_ERR_COINCIDENT: return "coincident distinct points";
        case SE_ERR_TOL_UNREACHABLE: return "tolerance unreachable at the requested precision";
        case SE_ERR_NOMEM: return "device allocation failed";
        case SE_ERR_HIP: return "HIP runtime error";
        case SE_ERR_STATE: return "call out of order";
        case SE_ERR_SCRATCH: return "input larger than the fixed scratch of an allocation-free call";
        default: return "unknown status";
    }
}

// Transform-size limits of the LDS-resident line FFTs.
static bool fft_sizes_ok(const int32_t* N, int ncomp, bool fp32)
{
    std::vector<int> rr;
    const int n[3] = {N[0], N[1], N[2]};
    return (n[0] % 2 == 0) && se_smooth_factors(n[0] / 2, &rr) && n[0] / 2 <= SE_FFT_LDS_ELEMS &&
           se_smooth_factors(n[1], &rr) && n[1] <= SE_FFT_LDS_ELEMS && se_smooth_factors(n[2], &rr) &&
           n[2] <= SE_FFT_LDS_ELEMS && se_fft_fits(n, ncomp, fp32);
}

static se_status validate_problem(const se_problem* prob)
{
    if (prob->struct_size != (int32_t)sizeof(se_problem)) return SE_ERR_ARG;
    if (prob->periodicity < 0 || prob->periodicity > 3) return SE_ERR_ARG;
    if (prob->kernel < SE_STOKESLET || prob->kernel > SE_HARMONIC) return SE_ERR_ARG;
    if (prob->tol_kind != SE_TOL_REL && prob->tol_kind != SE_TOL_ABS) return SE_ERR_ARG;
    if (!(prob->tol > 0) || !std::isfinite(prob->tol)) return SE_ERR_ARG;
    for (int i = 0; i < 3; i++)
        if (!(prob->box[i] > 0) || !std::isfinite(prob->box[i])) return SE_ERR_ARG;
    if (prob->n_src < 1 || prob->n_src > (int64_t)1 << 30) return SE_ERR_ARG;
    if (!prob->targets_are_sources && (prob->n_tgt < 1 || prob->n_tgt > (int64_t)1 << 30)) return SE_ERR_ARG;
    if (prob->n_rhs < 1) return SE_ERR_ARG;
    if (prob->precision < SE_PREC_AUTO || prob->precision > SE_PREC_FP32) return SE_ERR_ARG;
    if (prob->selector < SE_SELECT_ANALYTIC || prob->selector > SE_SELECT_MANUAL) return SE_ERR_ARG;
    if (prob->pollution != SE_POLLUTION_PAPER && prob->pollution != SE_POLLUTION_FINE) return SE_ERR_ARG;
    if (prob->window != SE_WINDOW_PKB && prob->window != SE_WINDOW_TG) return SE_ERR_ARG;
    return SE_OK;
}

se_status se_params_select(const se_problem* prob, se_params* out)
{
    if (!prob || !out) return SE_ERR_ARG;
    se_status st = validate_problem(prob);
    if (st != SE_OK) return st;
    if (prob->selector == SE_SELECT_MANUAL) return SE_ERR_ARG;
    std::string msg;
    if (prob->selector == SE_SELECT_LEARNED) return se_select_learned(prob, out, &msg);
    return se_select_params(prob, nullptr, out, &msg);
}

se_status se_plan_create(const se_problem* prob, const se_params* manual, se_plan** out)
{
    if (!prob || !out) return SE_ERR_ARG;
    *out = nullptr;
    {
        se_status st0 = validate_problem(prob);
        if (st0 != SE_OK) return st0;
    }

    se_plan* p = new (std::nothrow) se_plan();
    if (!p) return SE_ERR_NOMEM;
    p->prob = *prob;
    p->D = prob->periodicity;
    p->kernel = prob->kernel;
    p->ncomp = prob->kernel == SE_STRESSLET ? 6 : 3;
    p->nrhs = prob->n_rhs;
    // pairs of right-hand sides share the window weights, candidate lists and
    // real-space radial functions (6 gridded components, as for one stresslet)
    p->rb = (p->ncomp == 3 && p->nrhs >= 2) ? 2 : 1;
    p->device = prob->device;
    p->ns = prob->n_src;
    p->tas = prob->targets_are_sources != 0;
    p->nt = p->tas ? prob->n_src : prob->n_tgt;

    std::string msg;
    se_status st = prob->selector == SE_SELECT_LEARNED ? se_select_learned(prob, &p->par, &msg)
                                                       : se_select_params(prob, manual, &p->par, &msg);
    if (st != SE_OK) {
        delete p;
        return st;
    }
    // precision: the FP32 grid path is for rms-relative tolerances >= 1e-6.
    // An absolute tolerance is taken relative to the Fourier-part rms
    // estimate U of the selected parameters, the scale the relative form is
    // mapped through; without an estimate it counts as unreachable in FP32.
    {
        const double rel = prob->tol_kind == SE_TOL_REL ? prob->tol
                           : (p->par.U > 0.0 ? prob->tol / p->par.U : 0.0);
        if (prob->precision == SE_PREC_FP32) {
            if (!(rel >= 1e-6)) {
                delete p;
                return SE_ERR_TOL_UNREACHABLE;
            }
            p->fp32 = true;
        } else if (prob->precision == SE_PREC_AUTO) {
            p->fp32 = rel >= 1e-6;
        }
    }
    if (prob->selector == SE_SELECT_LEARNED && !fft_sizes_ok(p->par.n_fft, p->ncomp, p->fp32)) {
        st = se_select_params(prob, nullptr, &p->par, &msg);
        msg = "learned selector: grid beyond the FFT limits; analytic parameters";
        if (st != SE_OK) {
            delete p;
            return st;
        }
    }
    p->msg = msg;
    const se_params& par = p->par;

    // grid geometry
    se_grid_geom& g = p->g;
    g.D = p->D;
    for (int d = 0; d < 3; d++) {
        g.Mg[d] = par.M[d];
        g.h[d] = par.h[d];
        g.invh[d] = 1.0 / par.h[d];
        g.L[d] = prob->box[d];
        g.periodic[d] = d < p->D;
        g.x0[d] = d < p->D ? 0.0 : -0.5 * par.dL[d];
        int B = (g.Mg[d] % 4 == 0) ? 4 : ((g.Mg[d] % 2 == 0) ? 2 : 1);
        g.B[d] = B;
        g.nb[d] = (g.Mg[d] + B - 1) / B;
        p->Nfft[d] = par.n_fft[d];
    }
    p->nbins = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
    p->Hx = p->Nfft[0] / 2 + 1;
    p->Hp = (p->Hx + 7) / 8 * 8;
    se_tile_shape(p->ncomp, p->fp32, p->tile);
    for (int d = 0; d < 3; d++) p->ntile[d] = (g.Mg[d] + p->tile[d] - 1) / p->tile[d];

    // transform-size limits of the LDS-resident line FFTs
    std::vector<int> rr;
    bool ok = fft_sizes_ok(p->Nfft, p->ncomp, p->fp32);
    if (ok && (p->D == 1 || p->D == 2)) {
        aft_shapes(p);
        for (const se_aft_class& c : p->cls) {
            if (!c.active) continue;
            if (p->D == 1) ok = ok && se_smooth_factors(c.ny, &rr) && c.ny <= SE_FFT_LDS_ELEMS;
            ok = ok && se_smooth_factors(c.nz, &rr) && c.nz <= SE_FFT_LDS_ELEMS;
        }
    }
    if (ok && p->D == 0) {
        const int* n0 = p->par.n0_fft;
        ok = (n0[0] % 2 == 0) && se_smooth_factors(n0[0] / 2, &rr) && n0[0] / 2 <= SE_FFT_LDS_ELEMS &&
             se_smooth_factors(n0[1], &rr) && n0[1] <= SE_FFT_LDS_ELEMS && se_smooth_factors(n0[2], &rr) &&
             n0[2] <= SE_FFT_LDS_ELEMS;
    }
    if (!ok) {
        delete p;
        return SE_ERR_UNSUPPORTED;
    }

    if (hipSetDevice(p->device) != hipSuccess) {
        delete p;
        return SE_ERR_HIP;
    }
    // ---- allocation
    Alloc A{p};
    const size_t rs = p->fp32 ? sizeof(float) : sizeof(double);
    const int64_t nmax = std::max(p->ns, p->nt);
    p->d_flags = A.get<int>(1);
    p->d_src = A.get<double>(3 * p->ns);
    if (p->kernel == SE_STRESSLET) p->d_nrm = A.get<double>(3 * p->ns);
    p->d_src_perm = A.get<int>(p->ns);
    p->d_src_start = A.get<int>(p->nbins + 1);
    p->d_rwork = A.get<int>(p->nbins + 1);
    {
        const int64_t ntiles = (int64_t)p->ntile[0] * p->ntile[1] * p->ntile[2];
        p->d_rtx_s = A.get<int>(ntiles + 1);
        if (!p->tas) p->d_rtx_t = A.get<int>(ntiles + 1);
    }
    if (!p->tas) {
        p->d_tgt = A.get<double>(3 * p->nt);
        p->d_tgt_perm = A.get<int>(p->nt);
        p->d_tgt_start = A.get<int>(p->nbins + 1);
    }
    p->d_keys_a = A.get<int>(nmax);
    p->d_keys_b = A.get<int>(nmax);
    p->d_vals_a = A.get<int>(nmax);
    p->sort_tmp_bytes = se_sort_tmp_bytes(nmax, key_bits(p->nbins));
    p->d_sort_tmp = A.get<char>(std::max<size_t>(p->sort_tmp_bytes, 256));
    const size_t rb = (size_t)p->rb;
    p->d_fs = A.get<char>(rb * p->ncomp * p->ns * rs);
    p->d_fs64 = A.get<double>(rb * 4 * p->ns);
    p->d_red = A.get<double>(rb * (SE_RED_OUT + 7 * SE_RED_BLOCKS));
    const size_t gv = (size_t)g.Mg[0] * g.Mg[1] * g.Mg[2];
    p->d_grid = A.get<char>(rb * p->ncomp * gv * rs);
    const size_t sv = (size_t)p->Hp * p->Nfft[1] * g.Mg[2];
    p->d_spec = A.get<char>(rb * p->ncomp * sv * 2 * rs);
    p->d_pos4 = A.get<double>(4 * p->ns);
    if (!p->tas) p->d_tpos4 = A.get<double>(4 * p->nt);
    p->d_str4 = A.get<double>(rb * 4 * p->ns);
    if (p->kernel == SE_STRESSLET) p->d_nrm4 = A.get<double>(4 * p->ns);
    p->d_rtab = A.get<double>((size_t)2 * SE_RTAB_N * (SE_RTAB_DEG + 1));
    if (p->D == 0) p->d_ktab = A.get<double>((size_t)p->Hx * p->Nfft[1] * p->Nfft[2]);
    p->d_uF = A.get<double>(rb * 3 * p->nt);
    p->d_uR = A.get<double>(rb * 3 * p->nt);
    p->d_pkb = A.get<double>((size_t)par.P * (par.nu_deg + 1));
    p->d_invw2 = A.get<double>((size_t)p->Hx + p->Nfft[1] + p->Nfft[2]);
    const int Nh = p->Nfft[0] / 2;
    const size_t ntw = (size_t)Nh + (Nh + 1) + p->Nfft[1] + p->Nfft[2];
    p->d_tw = A.get<double>(2 * ntw);
    for (se_aft_class& c : p->cls) {
        if (!c.active) continue;
        const size_t nel = (size_t)c.nkx * c.ny * c.nz;
        c.buf = A.get<char>(rb * p->ncomp * nel * 2 * rs);  // one set per slot
        c.kv = A.get<double>((size_t)c.nkx + c.ny + c.nz);
        c.iw = A.get<double>((size_t)c.nkx + c.ny + c.nz);
        c.tw = A.get<double>(2 * ((size_t)1 + 2 + c.ny + c.nz));
        if (p->D == 1 && c.zero) c.mk = A.get<double>((size_t)2 * c.ny * c.nz);
    }
    if (!A.ok) {
        free_all(p);
        delete p;
        return SE_ERR_NOMEM;
    }

    // ---- host tables
    std::vector<double> pkb;
    se_pkb_coefficients(par.P, par.nu_deg, par.beta, &pkb);
    std::vector<double> iw;
    iw.reserve((size_t)p->Hx + p->Nfft[1] + p->Nfft[2]);
    for (int d = 0; d < 3; d++) {
        const int N = p->Nfft[d];
        const int cnt = d == 0 ? p->Hx : N;
        const double a = par.h[d] * par.P / 2.0;
        for (int i = 0; i < cnt; i++) {
            int kb = (d == 0) ? i : (i < N / 2 ? i : i - N);
            double k = 2.0 * M_PI * kb / (par.h[d] * N);
            double w = se_window_fourier(par, k, a);
            iw.push_back(1.0 / (w * w));
        }
    }
    std::vector<double> rtab;
    se_radial_table(se_rtab_xmax(par), &rtab);
    std::vector<double> tw;
    se_fft_twiddles(p->Nfft, &tw, p->tw_off);

    hipError_t e = hipMemcpy(p->d_pkb, pkb.data(), pkb.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_invw2, iw.data(), iw.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_rtab, rtab.data(), rtab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = aft_tables(p);
    if (e == hipSuccess) e = hipMemset(p->d_flags, 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(p->d_red, 0, rb * (SE_RED_OUT + 7 * SE_RED_BLOCKS) * sizeof(double));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(p);
        delete p;
        return SE_ERR_HIP;
    }
    if (p->D == 0) {
        se_status st0 = se_d0_precompute(p);
        if (st0 != SE_OK) {
            free_all(p);
            delete p;
            return st0;
        }
    }
    *out = p;
    return SE_OK;
}

void se_plan_destroy(se_plan* plan)
{
    if (!plan) return;
    hipSetDevice(plan->device);
    hipDeviceSynchronize();
    for (auto& e : plan->ev)
        if (e) hipEventDestroy(e);
    free_all(plan);
    delete plan;
}

se_status se_plan_get_params(const se_plan* plan, se_params* out)
{
    if (!plan || !out) return SE_ERR_ARG;
    *out = plan->par;
    return SE_OK;
}

size_t se_plan_workspace_bytes(const se_plan* plan) { return plan ? plan->ws_bytes : 0; }

const char* se_plan_last_message(const se_plan* plan) { return plan ? plan->msg.c_str() : ""; }

namespace {
struct PhaseScope {
    se_plan* p;
    int ph;
    hipStream_t s;
    PhaseScope(se_plan* p_, int ph_, hipStream_t s_) : p(p_), ph(ph_), s(s_)
    {
        if (p->timing) hipEventRecord(p->ev[2 * ph], s);
    }
    ~PhaseScope()
    {
        if (p->timing) hipEventRecord(p->ev[2 * ph + 1], s);
    }
};

void collect_phases(se_plan* p, const int* phases, int n)
{
    if (!p->timing) return;
    hipEventSynchronize(p->ev[2 * phases[n - 1] + 1]);
    for (int i = 0; i < n; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev[2 * phases[i]], p->ev[2 * phases[i] + 1]) == hipSuccess) {
            p->phase_ms[phases[i]] += ms;
            p->phase_n[phases[i]] += 1;
        }
    }
}
}  // namespace

se_status se_plan_set_timing(se_plan* plan, int32_t on)
{
    if (!plan) return SE_ERR_ARG;
    if (hipSetDevice(plan->device) != hipSuccess) return SE_ERR_HIP;
    if (on) {
        for (auto& e : plan->ev)
            if (!e && hipEventCreate(&e) != hipSuccess) return SE_ERR_HIP;
        for (int i = 0; i < SE_NUM_PHASES; i++) {
            plan->phase_ms[i] = 0.0;
            plan->phase_n[i] = 0;
        }
    }
    plan->timing = on != 0;
    return SE_OK;
}

se_status se_plan_phase_times(const se_plan* plan, double* ms, int32_t* counts, int32_t n)
{
    if (!plan || n < 0 || (n > 0 && (!ms || !counts))) return SE_ERR_ARG;
    for (int i = 0; i < n && i < SE_NUM_PHASES; i++) {
        ms[i] = plan->phase_ms[i];
        counts[i] = plan->phase_n[i];
    }
    return SE_OK;
}

static se_status bind_points(se_plan* p, const double* xyz, int64_t n, int* perm, int* start, double* sorted,
                             double* sorted4, hipStream_t s)
{
    se_launch_bin_keys(p->g, xyz, n, p->d_keys_a, p->d_vals_a, p->d_flags, p->wrap, s);
    se_status st = se_sort_pairs_raw(p->d_sort_tmp, p->sort_tmp_bytes, p->d_keys_a, p->d_keys_b, p->d_vals_a, perm,
                                     n, key_bits(p->nbins), s);
    if (st != SE_OK) {
        p->msg = "radix sort failed";
        return st;
    }
    se_launch_cell_starts(p->d_keys_b, n, p->nbins, start, s);
    se_launch_gather_sorted(xyz, perm, n, p->g, sorted, sorted4, 1, p->wrap, s);
    return check_hip(p, hipGetLastError(), "bind_points");
}

se_status se_set_geometry(se_plan* plan, const double* src_xyz, const double* nrm_xyz, const double* tgt_xyz,
                          void* stream)
{
    if (!plan || !src_xyz) return SE_ERR_ARG;
    if (plan->kernel == SE_STRESSLET && !nrm_xyz) return SE_ERR_ARG;
    if (!plan->tas && !tgt_xyz) return SE_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(plan->device) != hipSuccess) return SE_ERR_HIP;
    plan->have_geometry = false;
    se_status st;
    {
        PhaseScope ps(plan, 0, s);
        st = bind_points(plan, src_xyz, plan->ns, plan->d_src_perm, plan->d_src_start, plan->d_src, plan->d_pos4, s);
        if (st != SE_OK) return st;
        if (plan->kernel == SE_STRESSLET)
            se_launch_gather_sorted(nrm_xyz, plan->d_src_perm, plan->ns, plan->g, plan->d_nrm, plan->d_nrm4, 0, 0, s);
        if (!plan->tas) {
            st = bind_points(plan, tgt_xyz, plan->nt, plan->d_tgt_perm, plan->d_tgt_start, plan->d_tgt, plan->d_tpos4,
                             s);
            if (st != SE_OK) return st;
        }
    }
    {
        const int ph[1] = {0};
        collect_phases(plan, ph, 1);
    }
    st = check_hip(plan, hipGetLastError(), "se_set_geometry");
    if (st == SE_OK) plan->have_geometry = true;
    return st;
}

se_status se_run_plan(se_plan* p, const double* strengths, double* u, double* ur, double* uf, hipStream_t s)
{
    if (!p || !strengths) return SE_ERR_ARG;
    if (!p->have_geometry) return SE_ERR_STATE;
    if (hipSetDevice(p->device) != hipSuccess) return SE_ERR_HIP;
    // chunks of rb right-hand sides: one slot each in the plan's buffers
    for (int r0 = 0; r0 < p->nrhs; r0 += p->rb) {
        const int nr = std::min(p->rb, p->nrhs - r0);
        {
            PhaseScope ps(p, 1, s);
            for (int k = 0; k < nr; k++) {
                se_launch_strengths(p, strengths + (size_t)(r0 + k) * p->ns * 3, k, s);
                se_launch_reductions(p, k, s);
            }
            se_launch_fill_double(p->d_uF, 0.0, (int64_t)nr * 3 * p->nt, s);
        }
        {
            PhaseScope ps(p, 2, s);
            if (r0 == 0) se_launch_tile_prep(p, s);
            se_launch_spread(p, 0, nr, s);
        }
        {
            PhaseScope ps(p, 3, s);
            for (int k = 0; k < nr; k++) se_launch_fft_xy_forward(p, k, s);
        }
        {
            PhaseScope ps(p, 4, s);
            for (int k = 0; k < nr; k++) se_launch_fft_z_scale(p, k, s);
        }
        {
            PhaseScope ps(p, 5, s);
            for (int k = 0; k < nr; k++) se_launch_fft_inverse(p, k, s);
        }
        {
            PhaseScope ps(p, 6, s);
            se_launch_gather(p, 0, nr, s);
        }
        {
            PhaseScope ps(p, 7, s);
            if (r0 == 0) se_launch_real_prep(p, s);
            se_launch_real_space(p, 0, nr, s);
        }
        {
            PhaseScope ps(p, 8, s);
            for (int k = 0; k < nr; k++) {
                const size_t o = (size_t)(r0 + k) * p->nt * 3;
                se_launch_finalize(p, k, u ? u + o : nullptr, ur ? ur + o : nullptr, uf ? uf + o : nullptr, s);
            }
        }
        const int ph[8] = {1, 2, 3, 4, 5, 6, 7, 8};
        collect_phases(p, ph, 8);
    }
    return check_hip(p, hipGetLastError(), "se_execute");
}

se_status se_execute(se_plan* plan, const double* strengths, double* u_out, void* stream)
{
    if (!u_out) return SE_ERR_ARG;
    return se_run_plan(plan, strengths, u_out, nullptr, nullptr, (hipStream_t)stream);
}

se_status se_execute_split(se_plan* plan, const double* strengths, double* u_real, double* u_fourier, void* stream)
{
    if (!u_real || !u_fourier) return SE_ERR_ARG;
    return se_run_plan(plan, strengths, nullptr, u_real, u_fourier, (hipStream_t)stream);
}

se_status se_plan_set_wrap(se_plan* plan, int32_t on)
{
    if (!plan || (on != 0 && on != 1)) return SE_ERR_ARG;
    plan->wrap = on;
    return SE_OK;
}

se_status se_plan_set_shape(se_plan* plan, int32_t real_tb, int32_t fft_cols, int32_t tile_items)
{
    if (!plan || real_tb < 0 || real_tb > 4 || fft_cols < 0 || fft_cols > 16) return SE_ERR_ARG;
    if (fft_cols & (fft_cols - 1)) return SE_ERR_ARG;
    if (tile_items < 0 || tile_items > SE_TILE_ITEMS_MAX) return SE_ERR_ARG;
    plan->shape_real_tb = real_tb;
    plan->shape_fft_cols = fft_cols;
    plan->shape_tile_items = tile_items;
    return SE_OK;
}

se_status se_plan_get_shape(const se_plan* plan, int32_t* real_tb, int32_t* fft_cols, int32_t* tile_items)
{
    if (!plan || !real_tb || !fft_cols || !tile_items) return SE_ERR_ARG;
    *real_tb = plan->shape_real_tb;
    *fft_cols = plan->shape_fft_cols;
    *tile_items = plan->shape_tile_items;
    return SE_OK;
}

se_status se_sync_status(se_plan* plan)
{
    if (!plan) return SE_ERR_ARG;
    if (hipSetDevice(plan->device) != hipSuccess) return SE_ERR_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return SE_ERR_HIP;
    int flags = 0;
    if (hipMemcpy(&flags, plan->d_flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SE_ERR_HIP;
    if (flags) hipMemset(plan->d_flags, 0, sizeof(int));
    if (flags & SE_FLAG_NONFINITE) return SE_ERR_NONFINITE;
    if (flags & SE_FLAG_OUT_OF_BOX) return SE_ERR_OUT_OF_BOX;
    if (flags & SE_FLAG_COINCIDENT) return SE_ERR_COINCIDENT;
    return SE_OK;
}

se_status se_debug_cell_list(const se_plan* plan, int32_t which, const int32_t** perm, const int32_t** cell_start,
                             int32_t* nbins_xyz, int32_t* cell_width)
{
    if (!plan || !perm || !cell_start || !nbins_xyz || !cell_width) return SE_ERR_ARG;
    if (which != 0 && which != 1) return SE_ERR_ARG;
    if (which == 1 && plan->tas) which = 0;
    *perm = which == 0 ? plan->d_src_perm : plan->d_tgt_perm;
    *cell_start = which == 0 ? plan->d_src_start : plan->d_tgt_start;
    for (int d = 0; d < 3; d++) {
        nbins_xyz[d] = plan->g.nb[d];
        cell_width[d] = plan->g.B[d];
    }
    return SE_OK;
}

}  // extern "C"
