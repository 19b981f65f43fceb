/*
 * reduced_oracle.c -- zero modes (k^P = 0) of the Fourier-space Ewald sums
 * for D = 2 and D = 1 (TEST INFRASTRUCTURE ONLY; shares nothing with the GPU
 * path).  Bagge & Tornberg, Appendix A.2 and Appendix B.2:
 *
 *   D = 2:  u(x) += 1/(L1 L2) sum_n Q^{2P,(0)}(z - z_n) . f_n
 *     rotlet    eq. (2p-rotlet-Q0)     2 pi erf(xi r3) [[0,1,0],[-1,0,0],[0,0,0]]
 *     stokeslet eq. (2p-stokeslet-Q0) -2 pi (2 r3 erf(xi r3) + e^{-xi^2 r3^2}/(sqrt(pi) xi)) diag(1,1,0)
 *     stresslet eq. (2p-stresslet-Q0) -4 pi (erf(xi r3) + xi r3 e^{-xi^2 r3^2}/sqrt(pi)) C
 *
 *   D = 1:  u(x) += 1/L1 sum_n Q^{1P,(0)}(y - y_n, z - z_n) . f_n
 *     rotlet    eq. (1p-rotlet-Q0), stokeslet eq. (1p-stokeslet-Q0) (gauge l_B = 1),
 *     stresslet eq. (1p-stresslet-Q0), with their rho -> 0 limits
 *     eqs. (1p-stokeslet-Q0-limit), (1p-stresslet-Q0-limit) and a zero rotlet.
 *
 *
 *   harmonic (per component): Q^{H,2P,(0)} of Appendix A.2 and Q^{H,1P,(0)}
 *   of Appendix B.2 with l_H = 1 (gauges -2 pi |z| and -2 log(rho), their
 *   xi -> infinity limits):
 *     D = 2:  -2 pi (r3 erf(xi r3) + e^{-xi^2 r3^2}/(sqrt(pi) xi))
 *     D = 1:  -(E1(xi^2 rho^2) + log(rho^2)), at rho = 0: euler + log(xi^2)
 *
 * The nonsingular modes (k^P != 0) are evaluated by the caller through the
 * trapezoidal rule of the defining integrals (see oracle/reduced.py).
 */
#include <math.h>
#include <stdlib.h>

#define OR_STOKESLET 0
#define OR_ROTLET 1
#define OR_STRESSLET 2
#define OR_HARMONIC 3

static const double OR_PI = 3.14159265358979323846264338327950288;
static const double OR_EULER = 0.57721566490153286060651209008240243;

/* Exponential integral E1(x), x > 0: power series for x <= 1, continued
 * fraction (modified Lentz) for x > 1. */
double oracle_e1(double x)
{
    if (x <= 1.0) {
        double sum = 0.0, term = 1.0;
        for (int k = 1; k < 200; k++) {
            term *= -x / k;
            double add = -term / k;
            sum += add;
            if (fabs(add) < 1e-18 * fabs(sum)) break;
        }
        return -OR_EULER - log(x) + sum;
    }
    /* E1(x) = e^{-x} / (x + 1/(1 + 1/(x + 2/(1 + 2/(x + ...))))) in the form
     * e^{-x} * 1/(x+1-) 1^2/(x+3-) 2^2/(x+5-) ... */
    double b = x + 1.0, c = 1.0 / 1e-300, d = 1.0 / b, h = d;
    for (int i = 1; i < 500; i++) {
        double an = -(double)i * i;
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return h * exp(-x);
}

/* phi_1 = 1 - e^{-V}, phi_2 = 1 - (1 + V) e^{-V} (series at small V) */
static double phi1_of(double V) { return -expm1(-V); }

static double phi2_of(double V)
{
    if (V < 0.1) {
        double s = 0.0, pw = V * V, fact = 2.0;
        for (int n = 2; n < 30; n++) {
            s += ((n & 1) ? -1.0 : 1.0) * (n - 1) * pw / fact;
            pw *= V;
            fact *= (n + 1);
        }
        return s;
    }
    return -expm1(-V) - V * exp(-V);
}

/* Zero-mode tensor applied to a source: out_j += sum Q_{jl(m)} f_l (nu_m). */
static void zero_mode_2p(int kernel, double xi, double r3, const double *f, const double *nu, double *out)
{
    double e = exp(-xi * xi * r3 * r3);
    if (kernel == OR_HARMONIC) {
        double c = -2.0 * OR_PI * (r3 * erf(xi * r3) + e / (sqrt(OR_PI) * xi));
        for (int j = 0; j < 3; j++) out[j] += c * f[j];
    } else if (kernel == OR_ROTLET) {
        double c = 2.0 * OR_PI * erf(xi * r3);
        out[0] += c * f[1];
        out[1] += -c * f[0];
    } else if (kernel == OR_STOKESLET) {
        double c = -2.0 * OR_PI * (2.0 * r3 * erf(xi * r3) + e / (sqrt(OR_PI) * xi));
        out[0] += c * f[0];
        out[1] += c * f[1];
    } else {
        double c = -4.0 * OR_PI * (erf(xi * r3) + xi * r3 * e / sqrt(OR_PI));
        /* C_1lm: (1,3),(3,1); C_2lm: (2,3),(3,2); C_3lm: identity */
        out[0] += c * (f[0] * nu[2] + f[2] * nu[0]);
        out[1] += c * (f[1] * nu[2] + f[2] * nu[1]);
        out[2] += c * (f[0] * nu[0] + f[1] * nu[1] + f[2] * nu[2]);
    }
}

static void zero_mode_1p(int kernel, double xi, double r2, double r3, const double *f, const double *nu,
                         double *out)
{
    double rho2 = r2 * r2 + r3 * r3;
    double rho = sqrt(rho2);
    double V = xi * xi * rho2;
    if (kernel == OR_HARMONIC) {
        double c = rho == 0.0 ? OR_EULER + log(xi * xi) : -(oracle_e1(V) + log(rho2));
        for (int j = 0; j < 3; j++) out[j] += c * f[j];
    } else if (kernel == OR_ROTLET) {
        if (rho == 0.0) return;
        double c = 2.0 * phi1_of(V) / rho;
        double t2 = r2 / rho, t3 = r3 / rho;
        /* [[0, t3, -t2], [-t3, 0, 0], [t2, 0, 0]] */
        out[0] += c * (t3 * f[1] - t2 * f[2]);
        out[1] += c * (-t3 * f[0]);
        out[2] += c * (t2 * f[0]);
    } else if (kernel == OR_STOKESLET) {
        if (rho == 0.0) {
            double c = OR_EULER + log(xi * xi) - 1.0;
            out[0] += 2.0 * c * f[0];
            out[1] += c * f[1];
            out[2] += c * f[2];
            return;
        }
        double p0 = oracle_e1(V) + log(rho2) + 1.0;
        double p1 = phi1_of(V);
        double t2 = r2 / rho, t3 = r3 / rho;
        out[0] += -2.0 * (p0 + p1) * f[0];
        out[1] += -((p0 + 2.0 * t3 * t3 * p1) * f[1] - 2.0 * t2 * t3 * p1 * f[2]);
        out[2] += -(-2.0 * t2 * t3 * p1 * f[1] + (p0 + 2.0 * t2 * t2 * p1) * f[2]);
    } else {
        if (rho == 0.0) return;
        double p1 = phi1_of(V), p2 = phi2_of(V);
        double t2 = r2 / rho, t3 = r3 / rho;
        double R = -4.0 / rho;
        /* symmetric Q_jlm; nonzero entries (indices 1-based in the paper) */
        double Q[3][3][3] = {{{0}}};
        double q112 = R * t2 * (2.0 * p1 - p2);
        double q113 = R * t3 * (2.0 * p1 - p2);
        double q222 = R * t2 * (3.0 * p1 - (t2 * t2 + 3.0 * t3 * t3) * p2);
        double q223 = R * t3 * (p1 - (t3 * t3 - t2 * t2) * p2);
        double q233 = R * t2 * (p1 - (t2 * t2 - t3 * t3) * p2);
        double q333 = R * t3 * (3.0 * p1 - (3.0 * t2 * t2 + t3 * t3) * p2);
        /* fill all permutations of each index triple */
        double val[6] = {q112, q113, q222, q223, q233, q333};
        int trip[6][3] = {{0, 0, 1}, {0, 0, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
        for (int t = 0; t < 6; t++) {
            int a = trip[t][0], b = trip[t][1], c = trip[t][2];
            Q[a][b][c] = Q[a][c][b] = Q[b][a][c] = Q[b][c][a] = Q[c][a][b] = Q[c][b][a] = val[t];
        }
        for (int j = 0; j < 3; j++)
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++) out[j] += Q[j][l][m] * f[l] * nu[m];
    }
}

/* u_m += zero-mode part for D in {1, 2} (see header). */
void oracle_zero_mode(int D, int kernel, const double *L, double xi, long ns, const double *xs,
                      const double *f, const double *nu, long nt, const double *xt, double *u)
{
    double area = (D == 2) ? L[0] * L[1] : L[0];
#pragma omp parallel for schedule(static)
    for (long m = 0; m < nt; m++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long n = 0; n < ns; n++) {
            const double *fn = f + 3 * n;
            const double *nn = nu ? nu + 3 * n : NULL;
            if (D == 2)
                zero_mode_2p(kernel, xi, xt[3 * m + 2] - xs[3 * n + 2], fn, nn, acc);
            else
                zero_mode_1p(kernel, xi, xt[3 * m + 1] - xs[3 * n + 1], xt[3 * m + 2] - xs[3 * n + 2], fn, nn, acc);
        }
        for (int j = 0; j < 3; j++) u[3 * m + j] += acc[j] / area;
    }
}
