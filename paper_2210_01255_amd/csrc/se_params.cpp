// se_params.cpp -- parameter selection (Bagge & Tornberg, Sec. 4) and the
// window tables (Sec. 3.3).  Host code.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "se_internal.h"

namespace {

const double kPi = 3.14159265358979323846;

// Expected number of sources within r_c for the uniform system, Table 3
// (complexity-optimal-pts): rows S/Omega and T, columns D = 0..3.
const double kNrcUniform[2][4] = {{2500.0, 950.0, 450.0, 400.0}, {6000.0, 1600.0, 800.0, 800.0}};

// Box-padding factor lambda, Table 2 (estimates-lambda).
double lambda_factor(int kernel, int D)
{
    if (D == 0) return kernel == SE_STOKESLET ? 2.2 : (kernel == SE_STRESSLET ? 2.4 : 1.5);  // H: as Omega
    return 2.4;
}

struct Box {
    double V, Lc;  // volume and cube-equivalent side V^(1/3)
};

// Fourier-part rms estimate U(L,Q,xi), eqs. (pot-mag-est-stokeslet/-stresslet/-rotlet)
// with the mean constants C_U of Table 1.
double pot_rms(int kernel, const Box& b, double Q, double xi)
{
    double t = xi * b.Lc;
    double sq = std::sqrt(Q);
    if (kernel == SE_STOKESLET) {
        double fu = (1.0 + 1.323e-2 * t + 2.469e-4 * t * t) * std::exp(-5.205 / (t * t));
        return 1.8 * sq * fu / b.Lc;
    }
    if (kernel == SE_STRESSLET) return 7.2 * sq * std::sqrt(t) / (b.Lc * b.Lc);
    if (kernel == SE_HARMONIC) {
        // harmonic: U^2 = (8Q/V) int_{k0}^inf e^{-k^2/(2 xi^2)} / k^2 dk over the
        // Fourier part of uncorrelated charges, k0 = 2 pi / Lc
        const double k0 = 2.0 * kPi / b.Lc, s = 1.0 / (std::sqrt(2.0) * xi);
        const double I = std::exp(-k0 * k0 * s * s) / k0 - std::sqrt(kPi) * s * std::erfc(k0 * s);
        return std::sqrt(8.0 * Q / b.V * std::max(I, 0.0));
    }
    return 2.4 * sq * std::sqrt(t) * std::exp(-11.60 / (t * t)) / (b.Lc * b.Lc);
}

// Real-space truncation estimates, eqs. (rs-trunc-est-stokeslet/-stresslet/-rotlet):
// E = pref(rc) exp(-xi^2 rc^2).
double rs_pref(int kernel, const Box& b, double Q, double xi, double rc)
{
    if (kernel == SE_STOKESLET) return std::sqrt(4.0 * Q * rc / b.V);
    if (kernel == SE_STRESSLET) return std::sqrt(112.0 * Q * std::pow(xi, 4) * rc * rc * rc / (9.0 * b.V));
    // harmonic: (4 pi Q/V) int_rc^inf erfc(xi r)^2 dr with erfc(x) ~ e^{-x^2}/(x sqrt(pi))
    if (kernel == SE_HARMONIC) return std::sqrt(Q / (b.V * rc * rc * rc)) / (xi * xi);
    return std::sqrt(8.0 * Q / (3.0 * b.V * rc));
}

// Fourier truncation estimates, eqs. (fs-trunc-est-rotlet/-stokeslet/-stresslet):
// E = pref(k) exp(-k^2/(4 xi^2)).
double fs_pref(int kernel, const Box& b, double Q, double xi, double k)
{
    if (kernel == SE_STOKESLET) return 4.0 / (kPi * b.Lc) * std::sqrt(Q / 3.0);
    if (kernel == SE_STRESSLET) return 4.0 * k / (3.0 * kPi * b.Lc) * std::sqrt(7.0 * Q / 2.0);
    // harmonic: (8Q/V) int_k^inf e^{-k^2/(2 xi^2)} / k^2 dk ~ (8Q/V) xi^2 e^{-k^2/(2 xi^2)} / k^3
    if (kernel == SE_HARMONIC) return std::sqrt(8.0 * Q / b.V) * xi / std::pow(k, 1.5);
    return std::sqrt(8.0 * xi * xi * Q / (3.0 * kPi * b.V * k));
}

// Solve pref(rc) exp(-xi^2 rc^2) = tau for rc on the decaying branch.
double solve_rc(int kernel, const Box& b, double Q, double xi, double tau)
{
    double rc = 3.0 / xi;
    for (int it = 0; it < 200; it++) {
        double arg = rs_pref(kernel, b, Q, xi, rc) / tau;
        double nrc = arg > 1.0 ? std::sqrt(std::log(arg)) / xi : 0.5 / xi;
        if (std::fabs(nrc - rc) < 1e-15 * rc) {
            rc = nrc;
            break;
        }
        rc = nrc;
    }
    return rc;
}

// Solve pref(k) exp(-k^2/(4 xi^2)) = tau for k.
double solve_kinf(int kernel, const Box& b, double Q, double xi, double tau)
{
    double k = 8.0 * xi;
    for (int it = 0; it < 200; it++) {
        double arg = fs_pref(kernel, b, Q, xi, k) / tau;
        double nk = arg > 1.0 ? 2.0 * xi * std::sqrt(std::log(arg)) : 2.0 * xi;
        if (std::fabs(nk - k) < 1e-15 * k) {
            k = nk;
            break;
        }
        k = nk;
    }
    return k;
}

}  // namespace

// Factor n into radices from {8, 4, 2, 3, 5, 7} (largest first for the
// power-of-two part).  Returns false if n has another prime factor.
bool se_smooth_factors(int n, std::vector<int>* radices)
{
    radices->clear();
    if (n < 1) return false;
    int m = n;
    while (m % 8 == 0) {
        radices->push_back(8);
        m /= 8;
    }
    while (m % 4 == 0) {
        radices->push_back(4);
        m /= 4;
    }
    while (m % 2 == 0) {
        radices->push_back(2);
        m /= 2;
    }
    for (int r : {3, 5, 7}) {
        while (m % r == 0) {
            radices->push_back(r);
            m /= r;
        }
    }
    return m == 1;
}

// Stage order of the line FFTs: the smooth factors with the largest odd
// radix, if any, moved to the front.  The first Stockham stage writes each
// butterfly's outputs RAD elements apart, so consecutive work items store
// 16 * RAD bytes apart: for RAD = 8 (4) that is every (every other) 128-byte
// bank row, an 8-way (4-way) LDS bank conflict, while an odd RAD spreads
// them over all banks; later stages write runs of Ns >= RAD consecutive
// elements.  The kernels' radix codes and the twiddle tables both follow it.
bool se_fft_radix_order(int n, std::vector<int>* radices)
{
    if (!se_smooth_factors(n, radices)) return false;
    std::vector<int>& r = *radices;
    int odd = -1;
    for (int i = 0; i < (int)r.size(); i++)
        if ((r[i] & 1) && (odd < 0 || r[i] > r[odd])) odd = i;
    if (odd > 0) std::rotate(r.begin(), r.begin() + odd, r.begin() + odd + 1);
    return true;
}

namespace {

bool is_smooth(int n)
{
    std::vector<int> r;
    return se_smooth_factors(n, &r);
}

// Smallest n >= target that is a multiple of fM and whose FFT length
// (n/2 for an R2C axis when half=true) is 7-smooth.
int round_grid(double target, int fM, bool half)
{
    int n = fM * (int)std::ceil(target / fM - 1e-12);
    if (n < fM) n = fM;
    while (!(is_smooth(n) && (!half || is_smooth(n / 2)))) n += fM;
    return n;
}

long double bessel_i0(long double x)
{
    long double term = 1.0L, sum = 1.0L, q = x * x / 4.0L;
    for (int k = 1; k < 500; k++) {
        term *= q / ((long double)k * k);
        sum += term;
        if (term < sum * 1e-21L) break;
    }
    return sum;
}

}  // namespace

// Kaiser-Bessel window w0(r) = I0(beta sqrt(1-(r/a)^2))/I0(beta) on |r| <= a,
// eq. (KB-window), and its Fourier transform evaluated in FP64.
double se_kb_fourier(double k, double a, double beta)
{
    long double i0b = bessel_i0((long double)beta);
    long double s = (long double)beta * beta - (long double)k * k * a * a;
    long double val;
    if (s > 0) {
        long double r = std::sqrt(s);
        val = 2.0L * a * std::sinh(r) / (i0b * r);
    } else if (s < 0) {
        long double r = std::sqrt(-s);
        val = 2.0L * a * std::sin(r) / (i0b * r);
    } else {
        val = 2.0L * a / i0b;
    }
    return (double)val;
}

double se_tg_alpha(int P) { return 0.91 * (kPi / 2.0) * P; }

// Fourier transform of the untruncated Gaussian exp(-alpha (r/a)^2), used in
// the scaling step of the truncated-Gaussian window (Sec. 5.3):
// sqrt(pi/alpha) a exp(-k^2 a^2 / (4 alpha)).
double se_ug_fourier(double k, double a, double alpha)
{
    return std::sqrt(kPi / alpha) * a * std::exp(-k * k * a * a / (4.0 * alpha));
}

double se_window_fourier(const se_params& par, double k, double a)
{
    return par.window == SE_WINDOW_TG ? se_ug_fourier(k, a, par.alpha) : se_kb_fourier(k, a, par.beta);
}

// PKB window (Sec. 3.3): on each of the P subintervals [l h, (l+1) h],
// l = -P/2 .. P/2-1, interpolate the KB window at nu+1 Chebyshev points of
// the first kind.  coef[q*(nu+1) + c] multiplies sigma^c, with
// sigma = 2 s - 1 and s in [0,1] the local coordinate within subinterval
// q = l + P/2 (monomial basis, evaluated by Horner).
void se_pkb_coefficients(int P, int nu, double beta, std::vector<double>* coef)
{
    int n = nu + 1;
    coef->assign((size_t)P * n, 0.0);
    long double i0b = bessel_i0((long double)beta);
    std::vector<long double> A(n * n), rhs(n), sig(n);
    for (int i = 0; i < n; i++) sig[i] = -std::cos((2.0L * i + 1.0L) * (long double)kPi / (2.0L * n));
    for (int q = 0; q < P; q++) {
        int l = q - P / 2;
        for (int i = 0; i < n; i++) {
            long double s = (sig[i] + 1.0L) / 2.0L;
            long double u = 2.0L * ((long double)l + s) / (long double)P;  // r / a
            long double arg = 1.0L - u * u;
            long double w = arg > 0 ? bessel_i0((long double)beta * std::sqrt(arg)) / i0b : 1.0L / i0b;
            rhs[i] = w;
            long double pw = 1.0L;
            for (int c = 0; c < n; c++) {
                A[i * n + c] = pw;
                pw *= sig[i];
            }
        }
        // Gaussian elimination with partial pivoting (long double)
        for (int c = 0; c < n; c++) {
            int piv = c;
            for (int r = c + 1; r < n; r++)
                if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
            if (piv != c) {
                for (int k = 0; k < n; k++) std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(rhs[c], rhs[piv]);
            }
            for (int r = c + 1; r < n; r++) {
                long double fct = A[r * n + c] / A[c * n + c];
                for (int k = c; k < n; k++) A[r * n + k] -= fct * A[c * n + k];
                rhs[r] -= fct * rhs[c];
            }
        }
        for (int c = n - 1; c >= 0; c--) {
            long double acc = rhs[c];
            for (int k = c + 1; k < n; k++) acc -= A[c * n + k] * rhs[k];
            rhs[c] = acc / A[c * n + c];
        }
        for (int c = 0; c < n; c++) (*coef)[(size_t)q * n + c] = (double)rhs[c];
    }
}

// Radial functions of the real-space kernels in x = xi r:
//   G(x) = erfc(x) + (2x/sqrt(pi)) e^{-x^2},   E(x) = e^{-x^2},
// (eqs. stokeslet-real, rotlet-real, stresslet-real are combinations of G/r
// and E), as piecewise polynomials on SE_RTAB_N intervals of [0, xmax]
// (xmax = xi rc: only pairs inside the cut-off are evaluated), each
// interpolating at SE_RTAB_DEG+1 Chebyshev points of the first kind; monomial
// basis in sigma = 2 s - 1 (s local in [0,1]).
// Layout tab[f][interval][SE_RTAB_DEG+1], f = 0: G, 1: E.
void se_radial_table(double xmax, std::vector<double>* tab)
{
    const int n = SE_RTAB_DEG + 1;
    tab->assign((size_t)2 * SE_RTAB_N * n, 0.0);
    const long double w = (long double)xmax / SE_RTAB_N;
    const long double sqpi = std::sqrt((long double)kPi);
    std::vector<long double> A(n * n), rhs(n), sig(n);
    for (int i = 0; i < n; i++) sig[i] = -std::cos((2.0L * i + 1.0L) * (long double)kPi / (2.0L * n));
    for (int f = 0; f < 2; f++)
        for (int iv = 0; iv < SE_RTAB_N; iv++) {
            for (int i = 0; i < n; i++) {
                long double x = w * (iv + (sig[i] + 1.0L) / 2.0L);
                long double e = std::exp(-x * x);
                rhs[i] = f == 0 ? std::erfc(x) + 2.0L * x * e / sqpi : e;
                long double pw = 1.0L;
                for (int c = 0; c < n; c++) {
                    A[i * n + c] = pw;
                    pw *= sig[i];
                }
            }
            for (int c = 0; c < n; c++) {
                int piv = c;
                for (int r = c + 1; r < n; r++)
                    if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
                if (piv != c) {
                    for (int k = 0; k < n; k++) std::swap(A[c * n + k], A[piv * n + k]);
                    std::swap(rhs[c], rhs[piv]);
                }
                for (int r = c + 1; r < n; r++) {
                    long double fct = A[r * n + c] / A[c * n + c];
                    for (int k = c; k < n; k++) A[r * n + k] -= fct * A[c * n + k];
                    rhs[r] -= fct * rhs[c];
                }
            }
            for (int c = n - 1; c >= 0; c--) {
                long double acc = rhs[c];
                for (int k = c + 1; k < n; k++) acc -= A[c * n + k] * rhs[k];
                rhs[c] = acc / A[c * n + c];
            }
            for (int c = 0; c < n; c++) (*tab)[((size_t)f * SE_RTAB_N + iv) * n + c] = (double)rhs[c];
        }
}

// Parameter selection, Sec. 4.6 (steps 1-7), with xi taken from n_rc
// (Sec. 5.2) when not given, a relative tolerance mapped through U
// (Sec. 4.2), the pollution rule eq. (error-pollution-fix), grid rounding
// eq. (grid-adjustment) to 7-smooth multiples of f_M, eq. (extended-grid-size),
// eq. (truncation-radius), eq. (upsampling-factor-s0),
// eqs. (upsampling-factor-sstar), (estimate-kbarstar).
se_status se_select_params(const se_problem* p, const se_params* manual, se_params* out,
                           std::string* msg)
{
    const int D = p->periodicity, kernel = p->kernel;
    Box b;
    b.V = p->box[0] * p->box[1] * p->box[2];
    b.Lc = std::cbrt(b.V);
    const double N = (double)p->n_src;
    const double Q = p->source_q > 0 ? p->source_q : 3.0 * N;
    const double safety = p->safety > 0 ? p->safety : 1.0;
    const int fM = 4;
    se_params par;
    std::memset(&par, 0, sizeof(par));
    par.struct_size = sizeof(se_params);
    par.f_M = fM;

    if (p->selector == SE_SELECT_MANUAL) {
        if (!manual) {
            *msg = "selector MANUAL needs an se_params argument";
            return SE_ERR_ARG;
        }
        par = *manual;
        par.struct_size = sizeof(se_params);
        if (par.f_M <= 0) par.f_M = fM;
        if (par.xi <= 0 || par.rc <= 0 || par.P < 2 || (par.P & 1) || par.P > SE_MAX_P) {
            *msg = "manual parameters: need xi > 0, rc > 0 and even 2 <= P <= 32";
            return SE_ERR_ARG;
        }
        if (par.beta <= 0) par.beta = 2.5 * par.P;
        par.window = p->window;
        if (par.window == SE_WINDOW_TG && par.alpha <= 0) par.alpha = se_tg_alpha(par.P);
        if (par.window != SE_WINDOW_TG) par.alpha = 0.0;
        if (par.nu_deg <= 0) par.nu_deg = std::min(par.P / 2 + 2, 10);
        if (par.nu_deg > SE_MAX_NU) par.nu_deg = SE_MAX_NU;
        if (D < 3) {
            // free directions: steps 5-7 from (xi, rc, P) and the periodic
            // grid M[0..D-1] (D = 0: the target spacing h[0]), as the
            // analytic procedure completes its own
            bool have_m = D > 0;
            for (int i = 0; i < D; i++) have_m = have_m && par.M[i] >= 2 && !(par.M[i] & 1);
            if (!have_m && !(par.h[0] > 0)) {
                *msg = "manual parameters for D < 3: need even periodic grid sizes M[0..D-1] (D = 0: h[0] > 0)";
                return SE_ERR_ARG;
            }
            const double ht = have_m ? p->box[0] / par.M[0] : par.h[0];
            int mp[3] = {par.M[0], par.M[1], par.M[2]};
            const int nu = par.nu_deg;
            const double alpha = par.alpha, beta = par.beta;
            se_status st = se_complete_params(p, par.xi, par.rc, ht, par.P, out, msg, have_m ? mp : nullptr);
            if (st != SE_OK) return st;
            out->nu_deg = nu;
            out->beta = beta;
            out->alpha = alpha;
            return SE_OK;
        }
        for (int i = 0; i < 3; i++) {
            if (par.M[i] < 2 || (par.M[i] & 1)) {
                *msg = "manual parameters: grid sizes must be even and >= 2";
                return SE_ERR_ARG;
            }
            par.h[i] = p->box[i] / par.M[i];
            par.L_ext[i] = p->box[i];
            par.dL[i] = 0;
            par.n_fft[i] = par.M[i];
        }
        par.U = pot_rms(kernel, b, Q, par.xi);
        par.tau_abs = p->tol_kind == SE_TOL_ABS ? p->tol / safety : p->tol * par.U / safety;
        *out = par;
        return SE_OK;
    }
    se_targets t;
    se_analytic_targets(p, &t);
    return se_complete_params(p, t.xi, t.rc, t.h_t, t.P, out, msg);
}

// Steps 1-5 of Sec. 4.6: xi (given, or from N_rc with the real-space
// estimate, Sec. 5.2), rc, the target grid spacing and the window support
// after the pollution rule.
void se_analytic_targets(const se_problem* p, se_targets* out)
{
    const int D = p->periodicity, kernel = p->kernel;
    Box b;
    b.V = p->box[0] * p->box[1] * p->box[2];
    b.Lc = std::cbrt(b.V);
    const double N = (double)p->n_src;
    const double Q = p->source_q > 0 ? p->source_q : 3.0 * N;
    const double safety = p->safety > 0 ? p->safety : 1.0;
    // ---- xi and tau_abs
    double xi = p->xi;
    auto tau_of = [&](double x) {
        return p->tol_kind == SE_TOL_ABS ? p->tol / safety : p->tol * pot_rms(kernel, b, Q, x) / safety;
    };
    if (xi <= 0) {
        double nrc = p->n_rc > 0 ? p->n_rc : kNrcUniform[kernel == SE_STRESSLET ? 1 : 0][D];
        double rc = std::cbrt(3.0 * nrc * b.V / (4.0 * kPi * N));
        xi = 10.0 / b.Lc;
        for (int it = 0; it < 200; it++) {
            double arg = rs_pref(kernel, b, Q, xi, rc) / tau_of(xi);
            double nxi = arg > 1.0 ? std::sqrt(std::log(arg)) / rc : 1.0 / rc;
            // a relative tolerance is mapped through the Fourier-part estimate
            // U, which underflows when xi Lc is tiny (an N_rc radius far beyond
            // the box for a handful of sources): keep the last xi at which the
            // mapped tolerance is positive
            if (!std::isfinite(nxi) || !(tau_of(nxi) > 0.0)) break;
            if (std::fabs(nxi - xi) < 1e-14 * xi) {
                xi = nxi;
                break;
            }
            xi = nxi;
        }
    }
    const double tau = tau_of(xi);

    // step 1: real-space cut-off
    const double rc = solve_rc(kernel, b, Q, xi, tau);
    // step 2: grid spacing from the Fourier truncation estimate
    double kinf = solve_kinf(kernel, b, Q, xi, tau);
    double h_est = kPi / kinf;
    // step 3: window support from 10 U exp(-2.5 P) = tau (PKB); the truncated
    // Gaussian decays as exp(-alpha) = exp(-0.91 (pi/2) P) at the support edge
    // and takes the same form of estimate with that rate
    const double rate = p->window == SE_WINDOW_TG ? se_tg_alpha(1) : 2.5;
    double P_est = std::log(10.0 * pot_rms(kernel, b, Q, xi) / tau) / rate;
    if (P_est < 0) P_est = 0;
    // step 4: pollution rule
    const bool fine = D == 0 || p->pollution == SE_POLLUTION_FINE;
    double h_t = fine ? h_est / 1.1 : h_est / 1.05;
    double P_t = fine ? P_est + 2.0 : P_est + 4.0;
    // step 5: even window support
    int P = 2 * (int)std::ceil(P_t / 2.0 - 1e-12);
    if (P < 4) P = 4;
    out->xi = xi;
    out->rc = rc;
    out->h_t = h_t;
    out->P = P;
}

// Steps 5-7 of Sec. 4.6 from (xi, rc, target spacing h_t, window support P):
// KB shape and PKB degree, grid rounding eq. (grid-adjustment), the extended
// grid of the free directions eq. (extended-grid-size), the truncation radius
// eq. (truncation-radius), the upsampling factors eqs. (upsampling-factor-s0),
// (upsampling-factor-sstar), (estimate-kbarstar), and the three truncation
// estimates at the final parameters.
se_status se_complete_params(const se_problem* p, double xi, double rc, double h_t, int P, se_params* out,
                             std::string* msg, const int* M_periodic)
{
    const int D = p->periodicity, kernel = p->kernel;
    Box b;
    b.V = p->box[0] * p->box[1] * p->box[2];
    b.Lc = std::cbrt(b.V);
    const double N = (double)p->n_src;
    const double Q = p->source_q > 0 ? p->source_q : 3.0 * N;
    const double safety = p->safety > 0 ? p->safety : 1.0;
    const int fM = 4;
    if (!(xi > 0) || !(rc > 0) || !(h_t > 0) || !std::isfinite(xi) || !std::isfinite(rc) || !std::isfinite(h_t)) {
        *msg = "parameters: need finite xi, rc, h > 0";
        return SE_ERR_ARG;
    }
    if (P > SE_MAX_P) {
        *msg = "tolerance needs a window support above 32 grid points";
        return SE_ERR_TOL_UNREACHABLE;
    }
    se_params par;
    std::memset(&par, 0, sizeof(par));
    par.struct_size = sizeof(se_params);
    par.f_M = fM;
    const double U = pot_rms(kernel, b, Q, xi);
    const double tau = p->tol_kind == SE_TOL_ABS ? p->tol / safety : p->tol * U / safety;
    par.xi = xi;
    par.tau_abs = tau;
    par.U = U;
    par.rc = rc;
    par.P = P;
    par.beta = 2.5 * P;
    par.nu_deg = std::min(P / 2 + 2, 10);
    par.window = p->window;
    par.alpha = p->window == SE_WINDOW_TG ? se_tg_alpha(P) : 0.0;

    // periodic axes
    double h_common = h_t;
    for (int i = 0; i < D; i++) {
        int M = M_periodic ? M_periodic[i] : round_grid(p->box[i] / h_t, fM, i == 0);
        par.M[i] = M;
        par.h[i] = p->box[i] / M;
        par.L_ext[i] = p->box[i];
        par.dL[i] = 0.0;
        par.n_fft[i] = M;
        par.n0_fft[i] = M;
        par.nstar_fft[i] = M;
    }
    if (D > 0) {
        h_common = par.h[0];
        for (int i = 1; i < D; i++) h_common = std::min(h_common, par.h[i]);
    } else {
        // D = 0: h_actual = L/M_actual for the smallest side (eq. grid-adjustment)
        double Lmin = std::min(p->box[0], std::min(p->box[1], p->box[2]));
        int M = fM * (int)std::ceil(Lmin / h_t / fM - 1e-12);
        h_common = Lmin / M;
    }

    // step 6: extended grid in the free directions
    if (D < 3) {
        double lam = lambda_factor(kernel, D);
        double theta = (kernel == SE_ROTLET || kernel == SE_HARMONIC) ? 0.0 : 8.0;
        for (int i = D; i < 3; i++) {
            double target = p->box[i] / h_common + P + (lam - 1.0) * std::max((double)P, theta);
            // FFT lengths along free axes are s*M' (D=1,2) or 2M' (D=0); keep M' smooth
            int Mp = round_grid(target, fM, i == 0 && D == 0);
            par.M[i] = Mp;
            par.h[i] = h_common;
            par.L_ext[i] = h_common * Mp;
            par.dL[i] = par.L_ext[i] - p->box[i];
        }
        if (D == 2)
            par.R = par.L_ext[2];
        else if (D == 1)
            par.R = std::sqrt(par.L_ext[1] * par.L_ext[1] + par.L_ext[2] * par.L_ext[2]);
        else
            par.R = std::sqrt(par.L_ext[0] * par.L_ext[0] + par.L_ext[1] * par.L_ext[1] +
                              par.L_ext[2] * par.L_ext[2]);
        double Lmin = 1e300;
        for (int i = D; i < 3; i++) Lmin = std::min(Lmin, par.L_ext[i]);
        // step 7: upsampling
        double s0 = 1.0 + par.R / Lmin;
        s0 = std::ceil(10.0 * s0 - 1e-9) / 10.0;
        par.s0 = s0;
        double lnterm = std::log(U / (2.0 * tau));
        // eqs. (upsampling-factor-sstar), (estimate-kbarstar) are stated for a
        // cube; they follow from requiring |k^P| (s L'_i - L_i) >= log(U/(2E))
        // for the smallest |k^P| of a class, which for other boxes gives
        //   s_*  = max_i (L_i + max_j L_j log(U/2E)/(2 pi)) / L'_i   (free i),
        //   k*_j = ceil(L_j / min_i dL_i log(U/2E)/(2 pi) - 1)       (periodic j),
        // and the cube formulas when all sides are equal.
        double Lpmax = 0.0, dLmin = 1e300;
        for (int j = 0; j < D; j++) Lpmax = std::max(Lpmax, p->box[j]);
        for (int i = D; i < 3; i++) dLmin = std::min(dLmin, par.dL[i]);
        double sstar = 1.0;
        for (int i = D; i < 3; i++)
            sstar = std::max(sstar, (p->box[i] + Lpmax * lnterm / (2.0 * kPi)) / par.L_ext[i]);
        par.s_star = sstar;
        for (int j = 0; j < D && j < 2; j++) {
            int ks = (int)std::ceil(p->box[j] / dLmin * lnterm / (2.0 * kPi) - 1.0 - 1e-12);
            par.kstar[j] = std::max(ks, 0);
        }
        for (int i = D; i < 3; i++) {
            if (D == 0) {
                par.n_fft[i] = 2 * par.M[i];
                par.n0_fft[i] = round_grid(s0 * par.M[i], fM, i == 0);
                par.nstar_fft[i] = par.n_fft[i];
            } else {
                par.n_fft[i] = par.M[i];
                par.n0_fft[i] = round_grid(s0 * par.M[i], fM, false);
                par.nstar_fft[i] = round_grid(sstar * par.M[i], fM, false);
            }
        }
    }

    // estimates at the chosen parameters
    par.est_real = rs_pref(kernel, b, Q, xi, par.rc) * std::exp(-xi * xi * par.rc * par.rc);
    double kmin = 1e300;
    for (int i = 0; i < 3; i++) kmin = std::min(kmin, kPi / par.h[i]);
    par.est_fourier = fs_pref(kernel, b, Q, xi, kmin) * std::exp(-kmin * kmin / (4.0 * xi * xi));
    par.est_window = 10.0 * U * std::exp(p->window == SE_WINDOW_TG ? -par.alpha : -2.5 * P);
    *out = par;
    return SE_OK;
}
