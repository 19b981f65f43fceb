/*
 * ewald_oracle.c -- FP64 CPU reference for the Ewald-summed Stokes potentials.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU path: there is no grid, no window
 * function and no FFT in here.  It evaluates the potentials straight from the
 * paper's definitions (Bagge & Tornberg, "Fast Ewald summation for Stokes flow
 * with arbitrary periodicity"):
 *
 *   free-space kernels S, Omega, T ........ Sec. 2, eq. (stokes-kernels)
 *   harmonic kernel H = 1/|r| ............. Sec. 2, applied per component
 *                                            (three independent charge sets);
 *                                            Sec. 2.1 split with the classical
 *                                            screening, eq. (ewald-screening):
 *                                            real part erfc(xi r)/r, Fourier
 *                                            part (4 pi/k^2) gammaE
 *   real-space kernels S^R, Omega^R, T^R ... Sec. 2.1, eqs. (stokeslet-real),
 *                                            (rotlet-real), (stresslet-real)
 *   Fourier kernels (D = 3) ................ Sec. 2.1, eqs. (stokeslet-fourier),
 *                                            (rotlet-fourier), (stresslet-fourier)
 *   triply periodic Ewald sum .............. Sec. 2.2, eqs. (real-space-potential-3p),
 *                                            (fourier-space-potential-3p),
 *                                            (k0-stresslet-3p), (self-term),
 *                                            (3p-stokeslet-self-term)
 *   real-space part for any D .............. Sec. 2.3, eq. (real-space-potential-Dp)
 *   free space (D = 0) ..................... Sec. 2, eq. (periodic-potential) with
 *                                            the single image p = 0, summed directly
 *
 * Conventions: positions are row-major [n][3]; for the stokeslet and rotlet the
 * strengths are f[n][3]; for the stresslet the source is f_lm = q_l nu_m with
 * q[n][3] and nu[n][3].  No 1/(8 pi) prefactor (the paper's units).
 * self_src[m] is the index of the source that coincides with target m (the term
 * n = m, p = 0 that the starred sums omit), or -1.
 *
 * Plain loops; the only liberties are (a) skipping image shifts that cannot
 * lie within the cut-off radius, and (b) writing exp(-i k.x) as the product of
 * its three one-dimensional factors.  OpenMP splits independent targets.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

#define OR_STOKESLET 0
#define OR_ROTLET 1
#define OR_STRESSLET 2
#define OR_HARMONIC 3

static const double OR_PI = 3.14159265358979323846264338327950288;

static double kron(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Levi-Civita symbol epsilon_{abc} on indices 0,1,2 */
static double levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0.0;
    if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) ||
        (a == 2 && b == 0 && c == 1))
        return 1.0;
    return -1.0;
}

/* ------------------------------------------------------------------------ */
/* Free-space kernels, eq. (stokes-kernels):                                 */
/*   S_jl = delta_jl/|r| + r_j r_l/|r|^3                                     */
/*   Omega_jl = eps_jlm r_m/|r|^3                                            */
/*   T_jlm = -6 r_j r_l r_m/|r|^5                                            */
/* u_j += G . f  with the contractions of eq. (tensor-products).             */
/* ------------------------------------------------------------------------ */
void oracle_free_kernel(int kernel, const double *r, const double *f,
                        const double *nu, double *u)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = sqrt(r2);
    for (int j = 0; j < 3; j++) {
        double acc = 0.0;
        if (kernel == OR_STOKESLET) {
            for (int l = 0; l < 3; l++)
                acc += (kron(j, l) / rn + r[j] * r[l] / (rn * r2)) * f[l];
        } else if (kernel == OR_ROTLET) {
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++)
                    acc += levi(j, l, m) * r[m] / (rn * r2) * f[l];
        } else if (kernel == OR_HARMONIC) {
            acc = f[j] / rn;
        } else {
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++)
                    acc += -6.0 * r[j] * r[l] * r[m] / (rn * r2 * r2) * f[l] * nu[m];
        }
        u[j] += acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Real-space kernels, eqs. (stokeslet-real), (rotlet-real), (stresslet-real) */
/* ------------------------------------------------------------------------ */
void oracle_real_kernel(int kernel, double xi, const double *r, const double *f,
                        const double *nu, double *u)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = sqrt(r2);
    double ec = erfc(xi * rn);
    double gauss = exp(-xi * xi * r2);
    double sqpi = sqrt(OR_PI);
    for (int j = 0; j < 3; j++) {
        double acc = 0.0;
        if (kernel == OR_STOKESLET) {
            double c1 = ec / rn + 2.0 * xi * gauss / sqpi;
            double c2 = 4.0 * xi * gauss / sqpi;
            for (int l = 0; l < 3; l++)
                acc += ((kron(j, l) + r[j] * r[l] / r2) * c1 - kron(j, l) * c2) * f[l];
        } else if (kernel == OR_ROTLET) {
            double c1 = ec / rn + 2.0 * xi * gauss / sqpi;
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++)
                    acc += levi(j, l, m) * (r[m] / r2) * c1 * f[l];
        } else if (kernel == OR_HARMONIC) {
            acc = ec / rn * f[j];
        } else {
            double c1 = 3.0 * ec / rn + (3.0 + 2.0 * xi * xi * r2) * 2.0 * xi * gauss / sqpi;
            double c2 = 4.0 * xi * xi * xi * gauss / sqpi;
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++) {
                    double t = -2.0 * r[j] * r[l] * r[m] / (r2 * r2) * c1 +
                               (kron(j, l) * r[m] + kron(m, j) * r[l] + kron(l, m) * r[j]) * c2;
                    acc += t * f[l] * nu[m];
                }
        }
        u[j] += acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Real-space part, eq. (real-space-potential-Dp): sum over sources and over */
/* the image shifts p in P_DP (first D axes periodic) with |r| < rc, r =     */
/* x_m - x_n + p, skipping (n = self_src[m], p = 0).  Only image integers    */
/* whose shift can bring the pair inside rc are visited.                     */
/* Returns the number of coincident distinct pairs found (r = 0), which are  */
/* skipped.                                                                  */
/* ------------------------------------------------------------------------ */
long oracle_real_part(int D, int kernel, const double *L, double xi, double rc,
                      long ns, const double *xs, const double *f, const double *nu,
                      long nt, const double *xt, const long *self_src, double *u)
{
    long coincident = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : coincident)
    for (long m = 0; m < nt; m++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long n = 0; n < ns; n++) {
            double d[3];
            int lo[3], hi[3];
            for (int i = 0; i < 3; i++) {
                d[i] = xt[3 * m + i] - xs[3 * n + i];
                if (i < D) {
                    lo[i] = (int)ceil((-rc - d[i]) / L[i]) - 1;
                    hi[i] = (int)floor((rc - d[i]) / L[i]) + 1;
                } else {
                    lo[i] = 0;
                    hi[i] = 0;
                }
            }
            for (int p0 = lo[0]; p0 <= hi[0]; p0++)
                for (int p1 = lo[1]; p1 <= hi[1]; p1++)
                    for (int p2 = lo[2]; p2 <= hi[2]; p2++) {
                        double r[3] = {d[0] + p0 * L[0], d[1] + p1 * L[1], d[2] + p2 * L[2]};
                        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (r2 >= rc * rc) continue;
                        int p_is_zero = (p0 == 0 && p1 == 0 && p2 == 0);
                        if (p_is_zero && self_src && self_src[m] == n) continue;
                        if (r2 == 0.0) {
                            coincident++;
                            continue;
                        }
                        oracle_real_kernel(kernel, xi, r, f + 3 * n, nu ? nu + 3 * n : NULL, acc);
                    }
        }
        u[3 * m + 0] += acc[0];
        u[3 * m + 1] += acc[1];
        u[3 * m + 2] += acc[2];
    }
    return coincident;
}

/* ------------------------------------------------------------------------ */
/* Fourier-space Ewald kernels for D = 3 (k != 0).                           */
/* Returns A_j = sum_{l(,m)} Ghat^F_{jl(m)}(k) . S_{l(m)}  for a complex      */
/* structure factor S (3 entries for S/Omega, 9 entries [l][m] for T).       */
/*   Shat^F_jl = (-delta_jl k^2 + k_j k_l)(-8 pi/k^4) gammaH                 */
/*   Omegahat^F_jl = -eps_jlm i k_m (4 pi/k^2) gammaE                        */
/*   That^F_jlm = (-i(d_jl k_m + d_mj k_l + d_lm k_j) k^2 + 2i k_j k_l k_m)  */
/*                (-8 pi/k^4) gammaH                                         */
/* gammaE = exp(-k^2/(4 xi^2)), gammaH = gammaE (1 + k^2/(4 xi^2)),          */
/* eqs. (ewald-screening), (hasimoto-screening).                             */
/* ------------------------------------------------------------------------ */
static void fourier_kernel_apply(int kernel, double xi, const double *k,
                                 const double complex *S, double complex *A)
{
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double gE = exp(-k2 / (4.0 * xi * xi));
    double gH = gE * (1.0 + k2 / (4.0 * xi * xi));
    for (int j = 0; j < 3; j++) {
        double complex acc = 0.0;
        if (kernel == OR_STOKESLET) {
            for (int l = 0; l < 3; l++) {
                double G = (-kron(j, l) * k2 + k[j] * k[l]) * (-8.0 * OR_PI / (k2 * k2)) * gH;
                acc += G * S[l];
            }
        } else if (kernel == OR_ROTLET) {
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++) {
                    double complex G = -levi(j, l, m) * I * k[m] * (4.0 * OR_PI / k2) * gE;
                    acc += G * S[l];
                }
        } else if (kernel == OR_HARMONIC) {
            acc = (4.0 * OR_PI / k2) * gE * S[j];
        } else {
            for (int l = 0; l < 3; l++)
                for (int m = 0; m < 3; m++) {
                    double complex G =
                        (-I * (kron(j, l) * k[m] + kron(m, j) * k[l] + kron(l, m) * k[j]) * k2 +
                         2.0 * I * k[j] * k[l] * k[m]) *
                        (-8.0 * OR_PI / (k2 * k2)) * gH;
                    acc += G * S[3 * l + m];
                }
        }
        A[j] = acc;
    }
}

/* Enumerate k-bar in a half space with 0 < |k| <= kmax; k = 2 pi kbar_i / L_i. */
static long list_halfspace_k(const double *L, double kmax, const double *kbox, int D, int *Kb, int **out)
{
    /* kbox == NULL: the sphere |k| <= kmax; else the box |k_i| <= kbox[i] */
    for (int i = 0; i < 3; i++) Kb[i] = (int)floor((kbox ? kbox[i] : kmax) * L[i] / (2.0 * OR_PI));
    long cap = (long)(2 * Kb[0] + 1) * (2 * Kb[1] + 1) * (Kb[2] + 1);
    int *lst = (int *)malloc(sizeof(int) * 3 * (size_t)cap);
    long cnt = 0;
    for (int k3 = 0; k3 <= Kb[2]; k3++)
        for (int k2 = -Kb[1]; k2 <= Kb[1]; k2++)
            for (int k1 = -Kb[0]; k1 <= Kb[0]; k1++) {
                int upper = (k3 > 0) || (k3 == 0 && k2 > 0) || (k3 == 0 && k2 == 0 && k1 > 0);
                if (!upper) continue;
                /* D < 3: the modes with k^P = 0 are handled in closed form */
                if (D == 2 && k1 == 0 && k2 == 0) continue;
                if (D == 1 && k1 == 0) continue;
                double kk[3] = {2.0 * OR_PI * k1 / L[0], 2.0 * OR_PI * k2 / L[1],
                                2.0 * OR_PI * k3 / L[2]};
                double kn2 = kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2];
                if (!kbox && kn2 > kmax * kmax) continue;
                lst[3 * cnt + 0] = k1;
                lst[3 * cnt + 1] = k2;
                lst[3 * cnt + 2] = k3;
                cnt++;
            }
    *out = lst;
    return cnt;
}

/* one-dimensional phase factors e^{-i 2 pi kb x / L} for kb = -K..K */
static void phase_table(double x, double L, int K, double complex *E)
{
    for (int kb = -K; kb <= K; kb++) {
        double a = 2.0 * OR_PI * kb * x / L;
        E[kb + K] = cos(a) - I * sin(a);
    }
}

/* ------------------------------------------------------------------------ */
/* Fourier-space part for D = 3, eq. (fourier-space-potential-3p), k != 0,   */
/* truncated at |k| <= kmax:                                                 */
/*   u(x) = (1/|B|) sum_{k != 0} Ghat^F(k) . S(k) e^{i k.x},                 */
/*   S(k) = sum_n f_n e^{-i k.x_n}.                                          */
/* The terms k and -k are complex conjugates, so the half space is summed    */
/* and doubled (real part).  Returns the number of k-vectors used.           */
/*                                                                           */
/* With D = 2 or 1 the same sum over a cell whose free sides are L[i] = P_v  */
/* and with the k^P = 0 modes left out is the trapezoidal rule, step         */
/* 2 pi / P_v, of the integrals over the free wavenumbers in eqs.            */
/* (2p-fourier-space) / (1p-fourier-space) for the nonsingular modes.        */
/* ------------------------------------------------------------------------ */
static long fourier_sum(int D, int kernel, const double *L, double xi, double kmax, const double *kbox,
                        long ns, const double *xs, const double *f, const double *nu,
                        long nt, const double *xt, double *u)
{
    int Kb[3];
    int *kl = NULL;
    long nk = list_halfspace_k(L, kmax, kbox, D, Kb, &kl);
    int ncs = (kernel == OR_STRESSLET) ? 9 : 3;
    double complex *S = (double complex *)calloc((size_t)nk * ncs, sizeof(double complex));
    double V = L[0] * L[1] * L[2];

#pragma omp parallel
    {
        double complex *Sloc = (double complex *)calloc((size_t)nk * ncs, sizeof(double complex));
        double complex *E0 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[0] + 1));
        double complex *E1 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[1] + 1));
        double complex *E2 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[2] + 1));
#pragma omp for schedule(static)
        for (long n = 0; n < ns; n++) {
            phase_table(xs[3 * n + 0], L[0], Kb[0], E0);
            phase_table(xs[3 * n + 1], L[1], Kb[1], E1);
            phase_table(xs[3 * n + 2], L[2], Kb[2], E2);
            double src[9];
            if (kernel == OR_STRESSLET) {
                for (int l = 0; l < 3; l++)
                    for (int m = 0; m < 3; m++) src[3 * l + m] = f[3 * n + l] * nu[3 * n + m];
            } else {
                for (int l = 0; l < 3; l++) src[l] = f[3 * n + l];
            }
            for (long q = 0; q < nk; q++) {
                double complex ph = E0[kl[3 * q] + Kb[0]] * E1[kl[3 * q + 1] + Kb[1]] *
                                    E2[kl[3 * q + 2] + Kb[2]];
                for (int c = 0; c < ncs; c++) Sloc[q * ncs + c] += src[c] * ph;
            }
        }
#pragma omp critical
        {
            for (long i = 0; i < nk * ncs; i++) S[i] += Sloc[i];
        }
        free(Sloc);
        free(E0);
        free(E1);
        free(E2);
    }

    double complex *A = (double complex *)malloc(sizeof(double complex) * 3 * (size_t)nk);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nk; q++) {
        double kk[3] = {2.0 * OR_PI * kl[3 * q] / L[0], 2.0 * OR_PI * kl[3 * q + 1] / L[1],
                        2.0 * OR_PI * kl[3 * q + 2] / L[2]};
        fourier_kernel_apply(kernel, xi, kk, S + q * ncs, A + 3 * q);
    }

#pragma omp parallel
    {
        double complex *E0 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[0] + 1));
        double complex *E1 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[1] + 1));
        double complex *E2 = (double complex *)malloc(sizeof(double complex) * (2 * Kb[2] + 1));
#pragma omp for schedule(static)
        for (long m = 0; m < nt; m++) {
            /* e^{+i k.x} = conj(e^{-i k.x}) */
            phase_table(xt[3 * m + 0], L[0], Kb[0], E0);
            phase_table(xt[3 * m + 1], L[1], Kb[1], E1);
            phase_table(xt[3 * m + 2], L[2], Kb[2], E2);
            double acc[3] = {0.0, 0.0, 0.0};
            for (long q = 0; q < nk; q++) {
                double complex ph = conj(E0[kl[3 * q] + Kb[0]] * E1[kl[3 * q + 1] + Kb[1]] *
                                         E2[kl[3 * q + 2] + Kb[2]]);
                for (int j = 0; j < 3; j++) acc[j] += 2.0 * creal(A[3 * q + j] * ph);
            }
            for (int j = 0; j < 3; j++) u[3 * m + j] += acc[j] / V;
        }
        free(E0);
        free(E1);
        free(E2);
    }
    free(A);
    free(S);
    free(kl);
    return nk;
}

long oracle_fourier_part_3p(int kernel, const double *L, double xi, double kmax,
                            long ns, const double *xs, const double *f, const double *nu,
                            long nt, const double *xt, double *u)
{
    return fourier_sum(3, kernel, L, xi, kmax, NULL, ns, xs, f, nu, nt, xt, u);
}

/* The same lattice sum over the box |k_i| <= kbox[i] instead of a sphere:
 * the modes a grid of spacing h_i = pi/kbox[i] holds, the truncation the SE
 * method makes (Appendix C notes that it truncates a cube of side 2 k_inf
 * where its estimates assume a sphere). */
long oracle_fourier_part_3p_box(int kernel, const double *L, double xi, const double *kbox,
                                long ns, const double *xs, const double *f, const double *nu,
                                long nt, const double *xt, double *u)
{
    return fourier_sum(3, kernel, L, xi, 0.0, kbox, ns, xs, f, nu, nt, xt, u);
}

/* Nonsingular modes k^P != 0 for D = 2, 1; Lv = (L_1, L_2, P_v) or
 * (L_1, P_v, P_v) (see fourier_sum). */
long oracle_reduced_fourier_part(int D, int kernel, const double *Lv, double xi, double kmax,
                                 long ns, const double *xs, const double *f, const double *nu,
                                 long nt, const double *xt, double *u)
{
    return fourier_sum(D, kernel, Lv, xi, kmax, NULL, ns, xs, f, nu, nt, xt, u);
}

/* ------------------------------------------------------------------------ */
/* Non-periodic stresslet term of the triply periodic sum,                   */
/* eq. (k0-stresslet-3p):  u(x) = -(8 pi/|B|) sum_n (x - x_n)(q_n . nu_n).   */
/* ------------------------------------------------------------------------ */
void oracle_k0_stresslet_3p(const double *L, long ns, const double *xs, const double *q,
                            const double *nu, long nt, const double *xt, double *u)
{
    double V = L[0] * L[1] * L[2];
#pragma omp parallel for schedule(static)
    for (long m = 0; m < nt; m++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long n = 0; n < ns; n++) {
            double qn = q[3 * n] * nu[3 * n] + q[3 * n + 1] * nu[3 * n + 1] + q[3 * n + 2] * nu[3 * n + 2];
            for (int j = 0; j < 3; j++) acc[j] += (xt[3 * m + j] - xs[3 * n + j]) * qn;
        }
        for (int j = 0; j < 3; j++) u[3 * m + j] += -8.0 * OR_PI / V * acc[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Self term, eq. (self-term): -G^F(0; xi) . f(x_m); for the stokeslet this  */
/* is -4 xi/sqrt(pi) f (eq. 3p-stokeslet-self-term), zero for Omega and T;   */
/* for the harmonic H^F(0) = lim (1 - erfc(xi r))/r = 2 xi/sqrt(pi).         */
/* ------------------------------------------------------------------------ */
void oracle_self_part(int kernel, double xi, long nt, const long *self_src,
                      const double *f, double *u)
{
    if ((kernel != OR_STOKESLET && kernel != OR_HARMONIC) || !self_src) return;
    double c = kernel == OR_STOKESLET ? -4.0 * xi / sqrt(OR_PI) : -2.0 * xi / sqrt(OR_PI);
    for (long m = 0; m < nt; m++) {
        long n = self_src[m];
        if (n < 0) continue;
        for (int j = 0; j < 3; j++) u[3 * m + j] += c * f[3 * n + j];
    }
}

/* ------------------------------------------------------------------------ */
/* Free space, D = 0: eq. (periodic-potential) has the single image p = 0    */
/* and converges absolutely; sum it directly, omitting n = self_src[m].      */
/* ------------------------------------------------------------------------ */
long oracle_direct_0p(int kernel, long ns, const double *xs, const double *f, const double *nu,
                      long nt, const double *xt, const long *self_src, double *u)
{
    long coincident = 0;
#pragma omp parallel for schedule(static) reduction(+ : coincident)
    for (long m = 0; m < nt; m++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long n = 0; n < ns; n++) {
            if (self_src && self_src[m] == n) continue;
            double r[3] = {xt[3 * m] - xs[3 * n], xt[3 * m + 1] - xs[3 * n + 1],
                           xt[3 * m + 2] - xs[3 * n + 2]};
            if (r[0] == 0.0 && r[1] == 0.0 && r[2] == 0.0) {
                coincident++;
                continue;
            }
            oracle_free_kernel(kernel, r, f + 3 * n, nu ? nu + 3 * n : NULL, acc);
        }
        for (int j = 0; j < 3; j++) u[3 * m + j] += acc[j];
    }
    return coincident;
}

/* ------------------------------------------------------------------------ */
/* Brute-force image sum of eq. (periodic-potential) truncated to the        */
/* symmetric block |pbar_i| <= K over the first D axes.  Used only where the */
/* lattice sum converges absolutely (D = 1 rotlet and stresslet) or on tiny  */
/* inputs as a cross-check; never as the definition for D = 2, 3.            */
/* ------------------------------------------------------------------------ */
void oracle_image_block_sum(int D, int kernel, const double *L, int K, long ns,
                            const double *xs, const double *f, const double *nu, long nt,
                            const double *xt, const long *self_src, double *u)
{
    int lo[3], hi[3];
    for (int i = 0; i < 3; i++) {
        lo[i] = (i < D) ? -K : 0;
        hi[i] = (i < D) ? K : 0;
    }
#pragma omp parallel for schedule(static)
    for (long m = 0; m < nt; m++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int p0 = lo[0]; p0 <= hi[0]; p0++)
            for (int p1 = lo[1]; p1 <= hi[1]; p1++)
                for (int p2 = lo[2]; p2 <= hi[2]; p2++)
                    for (long n = 0; n < ns; n++) {
                        if (p0 == 0 && p1 == 0 && p2 == 0 && self_src && self_src[m] == n) continue;
                        double r[3] = {xt[3 * m] - xs[3 * n] + p0 * L[0],
                                       xt[3 * m + 1] - xs[3 * n + 1] + p1 * L[1],
                                       xt[3 * m + 2] - xs[3 * n + 2] + p2 * L[2]};
                        oracle_free_kernel(kernel, r, f + 3 * n, nu ? nu + 3 * n : NULL, acc);
                    }
        for (int j = 0; j < 3; j++) u[3 * m + j] += acc[j];
    }
}
