// Host-only exercise of the parameter planner (Sec. 4.6 and the window and
// radial-table set-up) for a sanitizer build: every kernel, periodicity,
// window, pollution rule and a spread of tolerances, box shapes and sizes.
// Prints one line per failed invariant and exits non-zero if any failed.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "se_internal.h"

static int fails = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            std::printf("FAIL %s: ", #c);               \
            std::printf(__VA_ARGS__);                   \
            std::printf("\n");                          \
            fails++;                                    \
        }                                               \
    } while (0)

int main()
{
    const double tols[] = {1e-3, 1e-6, 1e-9, 1e-12};
    const double boxes[][3] = {{1, 1, 1}, {3, 1, 1}, {1, 1, 2.5}, {1, 2, 1}};
    const long ns[] = {1, 100, 100000, 10000000};
    int selected = 0;
    for (int kernel = 0; kernel < 4; kernel++)
        for (int D = 0; D <= 3; D++)
            for (int window = 0; window < 2; window++)
                for (int pol = 0; pol < 2; pol++)
                    for (double tol : tols)
                        for (const auto& box : boxes)
                            for (long n : ns) {
                                se_problem p;
                                std::memset(&p, 0, sizeof p);
                                p.struct_size = sizeof p;
                                p.periodicity = D;
                                p.kernel = kernel;
                                p.tol_kind = SE_TOL_REL;
                                for (int i = 0; i < 3; i++) p.box[i] = box[i];
                                p.tol = tol;
                                p.precision = SE_PREC_FP64;
                                p.selector = SE_SELECT_ANALYTIC;
                                p.n_src = n;
                                p.targets_are_sources = 1;
                                p.n_rhs = 1;
                                p.pollution = pol;
                                p.window = window;
                                p.safety = 10.0;
                                se_params out;
                                std::memset(&out, 0, sizeof out);
                                out.struct_size = sizeof out;
                                std::string msg;
                                const se_status st = se_select_params(&p, nullptr, &out, &msg);
                                if (st != SE_OK) {
                                    CHECK(st == SE_ERR_TOL_UNREACHABLE || st == SE_ERR_UNSUPPORTED,
                                          "kernel %d D %d tol %g n %ld: status %d", kernel, D, tol, n, (int)st);
                                    continue;
                                }
                                selected++;
                                CHECK(out.P >= 2 && out.P % 2 == 0 && out.P <= 32, "P %d", out.P);
                                CHECK(out.xi > 0 && out.rc > 0 && std::isfinite(out.xi) && std::isfinite(out.rc),
                                      "xi %g rc %g", out.xi, out.rc);
                                for (int i = 0; i < 3; i++) {
                                    CHECK(out.M[i] >= 1 && out.n_fft[i] >= out.M[i] / 2, "axis %d M %d n_fft %d", i,
                                          out.M[i], out.n_fft[i]);
                                    std::vector<int> rad;
                                    CHECK(se_fft_radix_order(out.n_fft[i], &rad), "n_fft %d not smooth", out.n_fft[i]);
                                }
                                CHECK(out.est_real >= 0 && out.est_fourier >= 0 && out.est_window >= 0,
                                      "estimates %g %g %g", out.est_real, out.est_fourier, out.est_window);
                                se_targets t;
                                se_analytic_targets(&p, &t);
                                CHECK(t.xi > 0 && t.rc > 0 && t.h_t > 0 && t.P >= 2, "targets %g %g %g %d", t.xi,
                                      t.rc, t.h_t, t.P);
                                // completing the set's own (xi, rc, h, P) with its periodic grid
                                // sizes reproduces its grids
                                if (window == 0) {
                                    se_params m;
                                    std::memset(&m, 0, sizeof m);
                                    m.struct_size = sizeof m;
                                    std::string msg2;
                                    double ht = 1e300;
                                    for (int i = 0; i < 3; i++) ht = std::fmin(ht, out.h[i]);
                                    const se_status s2 = se_complete_params(&p, out.xi, out.rc, ht * (1.0 + 1e-12),
                                                                            out.P, &m, &msg2, out.M);
                                    CHECK(s2 == SE_OK, "completion status %d", (int)s2);
                                    if (s2 == SE_OK)
                                        for (int i = 0; i < D; i++)
                                            CHECK(m.M[i] == out.M[i], "periodic axis %d: %d vs %d", i, m.M[i],
                                                  out.M[i]);
                                }
                                std::vector<double> coef;
                                se_pkb_coefficients(out.P, out.nu_deg, out.beta, &coef);
                                CHECK(coef.size() == (size_t)out.P * (out.nu_deg + 1), "coefficients %zu",
                                      coef.size());
                                for (double c : coef) CHECK(std::isfinite(c), "coefficient %g", c);
                            }
    std::vector<double> tab;
    se_radial_table(6.0, &tab);
    for (double v : tab) CHECK(std::isfinite(v), "radial table %g", v);
    for (int n = 1; n <= 4096; n++) {
        std::vector<int> r;
        if (se_fft_radix_order(n, &r)) {
            long prod = 1;
            for (int x : r) prod *= x;
            CHECK(prod == n, "radices of %d multiply to %ld", n, prod);
        }
    }
    std::printf("planner check: %d parameter sets selected, %d failures\n", selected, fails);
    return fails ? 1 : 0;
}
