/* Host-only exercise of the oracle's C routines for a sanitizer build: every
 * kernel and periodicity on a small seeded input (sources = targets, so the
 * self-exclusion paths run), with a coincident pair for the direct sums.
 * Prints one line per non-finite result and exits non-zero if any. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

long oracle_real_part(int D, int kernel, const double *L, double xi, double rc, long ns, const double *xs,
                      const double *f, const double *nu, long nt, const double *xt, const long *self_src, double *u);
long oracle_fourier_part_3p(int kernel, const double *L, double xi, double kmax, long ns, const double *xs,
                            const double *f, const double *nu, long nt, const double *xt, double *u);
long oracle_reduced_fourier_part(int D, int kernel, const double *Lv, double xi, double kmax, long ns,
                                 const double *xs, const double *f, const double *nu, long nt, const double *xt,
                                 double *u);
void oracle_k0_stresslet_3p(const double *L, long ns, const double *xs, const double *q, const double *nu, long nt,
                            const double *xt, double *u);
void oracle_self_part(int kernel, double xi, long nt, const long *self_src, const double *f, double *u);
long oracle_direct_0p(int kernel, long ns, const double *xs, const double *f, const double *nu, long nt,
                      const double *xt, const long *self_src, double *u);
void oracle_image_block_sum(int D, int kernel, const double *L, int K, long ns, const double *xs, const double *f,
                            const double *nu, long nt, const double *xt, const long *self_src, double *u);
void oracle_zero_mode(int D, int kernel, const double *L, double xi, long ns, const double *xs, const double *f,
                      const double *nu, long nt, const double *xt, double *u);
double oracle_e1(double x);

static unsigned long long state = 0x2210012550ULL;
static double unif(void)
{
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int bad = 0;
static void check(const char *what, int D, int kernel, const double *u, long n)
{
    for (long i = 0; i < 3 * n; i++)
        if (!isfinite(u[i])) {
            printf("FAIL %s D=%d kernel=%d: u[%ld] = %g\n", what, D, kernel, i, u[i]);
            bad++;
            return;
        }
}

int main(void)
{
    enum { N = 24 };
    const double L[3] = {1.0, 1.3, 0.9};
    double xs[3 * N], f[3 * N], nu[3 * N], u[3 * N];
    long self[N];
    for (long i = 0; i < N; i++) {
        for (int d = 0; d < 3; d++) {
            xs[3 * i + d] = unif() * L[d];
            f[3 * i + d] = 2.0 * unif() - 1.0;
            nu[3 * i + d] = 2.0 * unif() - 1.0;
        }
        const double s = sqrt(nu[3 * i] * nu[3 * i] + nu[3 * i + 1] * nu[3 * i + 1] + nu[3 * i + 2] * nu[3 * i + 2]);
        for (int d = 0; d < 3; d++) nu[3 * i + d] /= s;
        self[i] = i;
    }
    const double xi = 6.0, rc = 0.45, kmax = 40.0;
    for (int kernel = 0; kernel < 4; kernel++) {
        for (int D = 0; D <= 3; D++) {
            memset(u, 0, sizeof u);
            oracle_real_part(D, kernel, L, xi, rc, N, xs, f, nu, N, xs, self, u);
            check("real part", D, kernel, u, N);
            if (D >= 1 && D <= 2) {
                memset(u, 0, sizeof u);
                oracle_reduced_fourier_part(D, kernel, L, xi, kmax, N, xs, f, nu, N, xs, u);
                check("reduced Fourier part", D, kernel, u, N);
                memset(u, 0, sizeof u);
                oracle_zero_mode(D, kernel, L, xi, N, xs, f, nu, N, xs, u);
                check("zero mode", D, kernel, u, N);
                memset(u, 0, sizeof u);
                oracle_image_block_sum(D, kernel, L, 2, N, xs, f, nu, N, xs, self, u);
                check("image block sum", D, kernel, u, N);
            }
        }
        memset(u, 0, sizeof u);
        oracle_fourier_part_3p(kernel, L, xi, kmax, N, xs, f, nu, N, xs, u);
        check("Fourier part", 3, kernel, u, N);
        memset(u, 0, sizeof u);
        oracle_self_part(kernel, xi, N, self, f, u);
        check("self part", 3, kernel, u, N);
        /* a coincident distinct pair: counted and skipped */
        double xc[3 * N];
        memcpy(xc, xs, sizeof xc);
        for (int d = 0; d < 3; d++) xc[3 + d] = xc[d];
        memset(u, 0, sizeof u);
        const long nc = oracle_direct_0p(kernel, N, xc, f, nu, N, xc, self, u);
        check("direct sum", 0, kernel, u, N);
        if (nc != 2) {
            printf("FAIL direct sum kernel=%d: %ld coincident pairs reported, 2 expected\n", kernel, nc);
            bad++;
        }
    }
    memset(u, 0, sizeof u);
    oracle_k0_stresslet_3p(L, N, xs, f, nu, N, xs, u);
    check("k = 0 stresslet", 3, 2, u, N);
    for (double x = 1e-6; x < 50.0; x *= 1.7)
        if (!(oracle_e1(x) > 0.0) || !isfinite(oracle_e1(x))) {
            printf("FAIL E1(%g) = %g\n", x, oracle_e1(x));
            bad++;
        }
    printf("oracle check: %d failures\n", bad);
    return bad ? 1 : 0;
}
