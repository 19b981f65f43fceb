// se_reference.cpp -- direct Ewald reference on the GPU (host driver).
// D = 3: classical Ewald sum (Sec. 2.2) with both truncations near e^{-42};
// D = 2, 1: the decomposition of Sec. 2.3 with the modes k^P != 0 of eqs.
// (2p-fourier-space) / (1p-fourier-space) as the trapezoidal rule in the
// free wavenumbers (the lattice sum over a cell extended by seven periodic
// lengths in the free directions) and the modes k^P = 0 in the closed forms
// of Appendices A.2 and B.2; D = 0: the free-space sum.  No grid and no
// window: used to check the fast method on every target of large systems.
#include <algorithm>
#include <cmath>
#include <vector>

#include "se_internal.h"

namespace {

const double kMargin = 6.5;  // xi rc and kmax / (2 xi): erfc(6.5), e^{-6.5^2} ~ 1e-19
const double kVirtual = 7.0; // free-direction padding of the virtual cell, in periodic lengths

}  // namespace

extern "C" se_status se_ewald_reference(int32_t kernel, int32_t periodicity, const double box[3], double xi,
                                        int64_t n_src, const double* src_xyz, const double* strengths,
                                        const double* normals_xyz, int64_t n_tgt, const double* tgt_xyz,
                                        double* u_out, int32_t device, void* stream)
{
    if (kernel < SE_STOKESLET || kernel > SE_HARMONIC) return SE_ERR_ARG;
    if (periodicity < 0 || periodicity > 3) return SE_ERR_ARG;
    if (!box || !src_xyz || !strengths || !u_out || n_src < 1 || n_src > ((int64_t)1 << 30)) return SE_ERR_ARG;
    if (kernel == SE_STRESSLET && !normals_xyz) return SE_ERR_ARG;
    const int tas = tgt_xyz ? 0 : 1;
    const int64_t nt = tas ? n_src : n_tgt;
    if (nt < 1 || nt > ((int64_t)1 << 30)) return SE_ERR_ARG;
    for (int d = 0; d < 3; d++)
        if (!(box[d] > 0) || !std::isfinite(box[d])) return SE_ERR_ARG;
    double Lmin = 1e300, Lmax = 0.0;  // over the periodic sides
    for (int d = 0; d < periodicity; d++) {
        Lmin = std::min(Lmin, box[d]);
        Lmax = std::max(Lmax, box[d]);
    }
    const double rc = periodicity > 0 ? 0.5 * Lmin : 0.0;
    if (periodicity > 0) {
        if (xi <= 0) xi = 2.0 * kMargin / Lmin;
        if (!std::isfinite(xi) || xi * rc < kMargin * (1.0 - 1e-12)) return SE_ERR_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) return SE_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    const double* xt = tas ? src_xyz : tgt_xyz;

    // the lattice cell: the box, with the free sides extended (D = 2, 1)
    double Lv[3];
    for (int d = 0; d < 3; d++) Lv[d] = d < periodicity ? box[d] : box[d] + kVirtual * Lmax;
    // half space of k: k1 > 0, or k1 = 0 and k2 > 0, or k1 = k2 = 0 and k3 > 0;
    // the modes k^P = 0 are left to the closed forms (D = 2, 1)
    std::vector<double> kv;
    if (periodicity > 0) {
        const double kmax = 2.0 * kMargin * xi;
        int K[3];
        for (int d = 0; d < 3; d++) K[d] = (int)std::ceil(kmax * Lv[d] / (2.0 * M_PI));
        for (int a = 0; a <= K[0]; a++)
            for (int b = -K[1]; b <= K[1]; b++)
                for (int c = -K[2]; c <= K[2]; c++) {
                    if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                    if ((periodicity == 2 && a == 0 && b == 0) || (periodicity == 1 && a == 0)) continue;
                    const double k[3] = {2.0 * M_PI * a / Lv[0], 2.0 * M_PI * b / Lv[1], 2.0 * M_PI * c / Lv[2]};
                    if (k[0] * k[0] + k[1] * k[1] + k[2] * k[2] > kmax * kmax) continue;
                    kv.insert(kv.end(), k, k + 3);
                }
    }
    const int nk = (int)(kv.size() / 3);
    double *d_kv = nullptr, *d_U = nullptr, *d_sums = nullptr;
    int* d_flags = nullptr;
    se_status st = SE_OK;
    auto ok = [&](hipError_t e) {
        if (e == hipErrorOutOfMemory) st = SE_ERR_NOMEM;
        else if (e != hipSuccess && st == SE_OK) st = SE_ERR_HIP;
        return st == SE_OK;
    };
    if (ok(hipMalloc(&d_flags, sizeof(int))) && ok(hipMalloc(&d_sums, 8 * sizeof(double))) &&
        (nk == 0 || (ok(hipMalloc(&d_kv, kv.size() * sizeof(double))) &&
                     ok(hipMalloc(&d_U, (size_t)nk * 6 * sizeof(double))))) &&
        (nk == 0 || ok(hipMemcpy(d_kv, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice))) &&
        ok(hipMemsetAsync(d_flags, 0, sizeof(int), s))) {
        se_launch_dref_real(kernel, periodicity, box, xi, rc, n_src, src_xyz, strengths, normals_xyz, nt, xt, tas,
                            u_out, d_flags, s);
        if (periodicity > 0) {
            se_launch_dref_kspace(kernel, nk, d_kv, xi, Lv[0] * Lv[1] * Lv[2], n_src, src_xyz, strengths,
                                  normals_xyz, d_U, nt, xt, u_out, s);
            se_launch_dref_zero(kernel, periodicity, box, xi, n_src, src_xyz, strengths, normals_xyz, nt, xt, u_out,
                                s);
            se_launch_dref_terms(kernel, periodicity, box, xi, n_src, src_xyz, strengths, normals_xyz, nt, xt, tas,
                                 d_sums, u_out, s);
        }
        int flags = 0;
        if (ok(hipGetLastError()) && ok(hipStreamSynchronize(s)) &&
            ok(hipMemcpy(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost)) && (flags & SE_FLAG_COINCIDENT))
            st = SE_ERR_COINCIDENT;
    }
    hipStreamSynchronize(s);
    for (void* q : {(void*)d_kv, (void*)d_U, (void*)d_sums, (void*)d_flags})
        if (q) hipFree(q);
    return st;
}
