// se_internal.h -- private declarations shared by the library's own sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/se.h"

#define SE_VERSION_MAJOR 0
#define SE_VERSION_MINOR 1
#define SE_VERSION_PATCH 0

// Device-side error flags (bit set, read by se_sync_status).
#define SE_FLAG_OUT_OF_BOX 1
#define SE_FLAG_NONFINITE 2
#define SE_FLAG_COINCIDENT 4

// Largest supported window support and polynomial degree.
// Kernels whose scalar building block is the harmonic (rotlet, harmonic)
// rather than the biharmonic, and kernels odd in k (no real Nyquist mode).
constexpr bool se_harmonic_based(int kernel) { return kernel == SE_ROTLET || kernel == SE_HARMONIC; }
constexpr bool se_odd_kernel(int kernel) { return kernel == SE_ROTLET || kernel == SE_STRESSLET; }

#define SE_MAX_P 32
#define SE_MAX_NU 10

// Real-space radial-function table (see se_radial_table)
#define SE_RTAB_N 32
#define SE_RTAB_DEG 10

// Source reductions: SE_RED_OUT results followed by 7 x SE_RED_BLOCKS partials.
#define SE_RED_OUT 8
#define SE_RED_BLOCKS 256

// Line FFT limits (LDS-resident lines).
#define SE_FFT_MAX_LEN 4096
#define SE_FFT_THREADS 256
#define SE_FFT_LDS_ELEMS 2048  // complex elements per workgroup in the line kernels

struct se_grid_geom {
    int D;
    int Mg[3];       // grid points per axis (periodic M_i, free M'_i)
    double x0[3];    // physical coordinate of grid point 0
    double h[3];
    double invh[3];
    double L[3];     // primary cell
    int periodic[3];
    int B[3];        // grid cells per bin
    int nb[3];       // bins per axis
};

// Per-axis FFT description for the R2C/C2C/C2R passes.
struct se_fft_axis {
    int n_in;    // valid input length (rest zero padded)
    int n_fft;   // transform length
    int n_out;   // outputs kept after the inverse transform
    std::vector<int> radices;  // factorisation of n_fft (or n_fft/2 on the R2C axis)
};

// One upsampled mode class of the adaptive Fourier transform (D = 1, 2):
// [0] the modes k^P = 0 (modified kernels, upsampling s0), [1] the set K_*
// (regular kernels, upsampling s_*).  The class data lives in its own buffer
// [c][nz][ny][nkx] (complex, grid precision), zero padded in the free
// directions, so plain line FFTs of the padded lengths apply.
struct se_aft_class {
    int active = 0;
    int zero = 0;            // 1: the k^P = 0 class
    int nkx = 0, ny = 0, nz = 0;
    int kx_lo = 0;           // main-spectrum kx index of local kx 0
    int ky_lo = 0;           // D = 2: signed ky index of local row 0
    void* buf = nullptr;
    double* kv = nullptr;    // wavenumbers [nkx | ny | nz]
    double* iw = nullptr;    // 1/what^2 [nkx | ny | nz]
    double* tw = nullptr;    // twiddles for the (ny, nz) line FFTs
    double* mk = nullptr;    // D = 1, k^P = 0: [ny*nz][2] = (Hhat_R, Bhat_R)
    int tw_off[4] = {0, 0, 0, 0};
    double scale = 0.0;      // h1 h2 h3 / (N1 N2 N3) with the class lengths
};

struct se_plan {
    se_problem prob{};
    se_params par{};
    int D = 3;
    int kernel = 0;
    int ncomp = 3;   // gridded components (3, or 6 for the symmetrised stresslet source)
    int nrhs = 1;
    int rb = 1;      // right-hand sides per chunk (buffers hold rb slots)
    int shape_real_tb = 0;   // launch-shape knobs (0: automatic), see se_plan_set_shape
    int wrap = 0;            // reduce periodic coordinates modulo L_i when binding (se_plan_set_wrap)
    int shape_fft_cols = 0;
    int shape_tile_items = 0;  // gridding/gathering work item: candidates in batches of 64 (0: automatic)
    bool fp32 = false;
    int device = 0;
    int64_t ns = 0, nt = 0;
    bool tas = true;
    se_grid_geom g{};
    int64_t nbins = 0;
    int Nfft[3] = {0, 0, 0};
    int Hx = 0;              // R2C half-spectrum extent along x
    int Hp = 0;              // half-spectrum row pitch (Hx rounded up to 8: 128-byte rows in FP64)
    int tile[3] = {16, 16, 8};  // spread/gather tile (grid points)
    int ntile[3] = {0, 0, 0};

    // device buffers
    int* d_flags = nullptr;
    double* d_src = nullptr;       // sorted sources, SoA [3][ns]
    double* d_nrm = nullptr;       // sorted normals, SoA [3][ns] (stresslet)
    int* d_src_perm = nullptr;     // sorted -> original
    int* d_src_start = nullptr;    // [nbins+1]
    double* d_tgt = nullptr;       // sorted targets SoA [3][nt] (null when tas)
    int* d_tgt_perm = nullptr;
    int* d_tgt_start = nullptr;
    int* d_keys_a = nullptr;       // sort scratch
    int* d_keys_b = nullptr;
    int* d_vals_a = nullptr;
    void* d_sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    void* d_fs = nullptr;          // sorted strengths in grid precision [ncomp][ns]
    double* d_fs64 = nullptr;      // sorted strengths FP64 [3][ns] (self term), q.nu [ns]
    double* d_red = nullptr;       // reductions: [0] sum q.nu, [1..3] sum x (q.nu), [4..6] sum f; partials
    void* d_grid = nullptr;        // real grid [ncomp][Mz][My][Mx]
    void* d_spec = nullptr;        // half spectrum [ncomp][Mz][Ny][Hp] complex
    double* d_pos4 = nullptr;      // sorted sources AoS [ns][4] (x, y, z, 0)
    double* d_tpos4 = nullptr;     // sorted targets AoS [nt][4] (null when tas)
    double* d_str4 = nullptr;      // sorted strengths AoS [ns][4] (f or q, 0)
    double* d_nrm4 = nullptr;      // sorted normals AoS [ns][4] (stresslet)
    double* d_rtab = nullptr;      // radial-function table
    int* d_rwork = nullptr;        // real-space work offsets: target chunks per block, scanned (nbins + 1)
    int* d_rtx_s = nullptr;        // gridding: items beyond each tile's first, scanned (ntiles + 1)
    int* d_rtx_t = nullptr;        // gathering at separate targets: the same (ntiles + 1)
    double* d_ktab = nullptr;      // D = 0: truncated kernel Ahat_{R,tr} on the half spectrum
    double* d_uF = nullptr;        // [3][nt] sorted order
    double* d_uR = nullptr;        // [3][nt]
    double* d_pkb = nullptr;       // PKB coefficients [P][nu+1]
    double* d_invw2 = nullptr;     // 1/what0(k)^2 per axis, concatenated [Nx/2+1 | Ny | Nz]
    double* d_tw = nullptr;        // twiddles (complex FP64), see se_fft layout
    se_aft_class cls[2];           // D = 1, 2 upsampled classes ([0] k^P = 0, [1] K_*)
    int tw_off[4] = {0, 0, 0, 0};  // offsets (complex elements) of x-half, x-post, y, z tables
    size_t ws_bytes = 0;
    bool timing = false;
    hipEvent_t ev[2 * SE_NUM_PHASES] = {};
    double phase_ms[SE_NUM_PHASES] = {};
    int phase_n[SE_NUM_PHASES] = {};
    bool have_geometry = false;
    std::string msg;
};

// Per-slot buffer views (a chunk of rb right-hand sides shares the geometry).
inline size_t se_grid_elems(const se_plan* p) { return (size_t)p->g.Mg[0] * p->g.Mg[1] * p->g.Mg[2]; }
inline size_t se_spec_elems(const se_plan* p) { return (size_t)p->Hp * p->Nfft[1] * p->g.Mg[2]; }
inline size_t se_real_bytes(const se_plan* p) { return p->fp32 ? sizeof(float) : sizeof(double); }
inline void* se_slot_grid(const se_plan* p, int slot)
{
    return (char*)p->d_grid + (size_t)slot * p->ncomp * se_grid_elems(p) * se_real_bytes(p);
}
inline void* se_slot_spec(const se_plan* p, int slot)
{
    return (char*)p->d_spec + (size_t)slot * p->ncomp * se_spec_elems(p) * 2 * se_real_bytes(p);
}
inline void* se_slot_fs(const se_plan* p, int slot)
{
    return (char*)p->d_fs + (size_t)slot * p->ncomp * p->ns * se_real_bytes(p);
}
inline double* se_slot_fs64(const se_plan* p, int slot) { return p->d_fs64 + (size_t)slot * 4 * p->ns; }
inline double* se_slot_str4(const se_plan* p, int slot) { return p->d_str4 + (size_t)slot * 4 * p->ns; }
inline double* se_slot_red(const se_plan* p, int slot) { return p->d_red + (size_t)slot * (SE_RED_OUT + 7 * SE_RED_BLOCKS); }
inline double* se_slot_uF(const se_plan* p, int slot) { return p->d_uF + (size_t)slot * 3 * p->nt; }
inline double* se_slot_uR(const se_plan* p, int slot) { return p->d_uR + (size_t)slot * 3 * p->nt; }

// ---- planner (se_params.cpp)
se_status se_select_params(const se_problem* p, const se_params* manual, se_params* out,
                           std::string* msg);
// M_periodic: the periodic axes' grid sizes to use instead of rounding
// box / h_t (manual parameters).
se_status se_complete_params(const se_problem* p, double xi, double rc, double h_t, int P, se_params* out,
                             std::string* msg, const int* M_periodic = nullptr);
// Steps 1-5 of the analytic procedure (before grid rounding and completion).
struct se_targets {
    double xi, rc, h_t;
    int P;
};
void se_analytic_targets(const se_problem* p, se_targets* out);
// Learned selection (MLP proposal, then completion and the estimate check);
// falls back to se_select_params and says so in msg.
se_status se_select_learned(const se_problem* p, se_params* out, std::string* msg);
bool se_smooth_factors(int n, std::vector<int>* radices);
bool se_fft_radix_order(int n, std::vector<int>* radices);
void se_pkb_coefficients(int P, int nu, double beta, std::vector<double>* coef);
// Truncated-Gaussian shape 0.91 (pi/2) P, the untruncated Gaussian's Fourier
// transform, and the transform of the plan's window (KB or UG) at k for
// half-support a.
double se_tg_alpha(int P);
double se_ug_fourier(double k, double a, double alpha);
double se_window_fourier(const se_params& par, double k, double a);
void se_radial_table(double xmax, std::vector<double>* tab);
// Range of the radial table: x = xi r for r < rc (slightly widened).
inline double se_rtab_xmax(const se_params& par) { return par.xi * par.rc * (1.0 + 1e-9) + 1e-300; }
double se_kb_fourier(double k, double a, double beta);

// ---- kernels (se_*.hip): host-side launch wrappers
void se_launch_fill_int(int* p, int v, int64_t n, hipStream_t s);
void se_launch_fill_double(double* p, double v, int64_t n, hipStream_t s);
void se_launch_fill_bytes_zero(void* p, size_t bytes, hipStream_t s);
void se_launch_bin_keys(const se_grid_geom& g, const double* xyz, int64_t n, int* keys, int* idx,
                        int* flags, int wrap, hipStream_t s);
void se_launch_gather_sorted(const double* xyz, const int* perm, int64_t n, const se_grid_geom& g,
                             double* out_soa, double* out_aos4, int sanitize, int wrap, hipStream_t s);
void se_launch_cell_starts(const int* sorted_keys, int64_t n, int64_t nbins, int* start,
                           hipStream_t s);
// Stable radix sort of (key, value) pairs, keys in [0, 2^end_bit) (se_geom.hip).
se_status se_sort_pairs_raw(void* tmp, size_t tmp_bytes, const int* keys_in, int* keys_out, const int* vals_in,
                            int* vals_out, int64_t n, int end_bit, hipStream_t s);
size_t se_sort_tmp_bytes(int64_t n, int end_bit);
void se_launch_strengths(const se_plan* p, const double* f, int slot, hipStream_t s);
void se_launch_spread(const se_plan* p, int slot0, int nslot, hipStream_t s);
void se_launch_fft_xy_forward(const se_plan* p, int slot, hipStream_t s);
void se_launch_fft_z_scale(const se_plan* p, int slot, hipStream_t s);
void se_launch_fft_inverse(const se_plan* p, int slot, hipStream_t s);
void se_launch_gather(const se_plan* p, int slot0, int nslot, hipStream_t s);
// Work offsets of the blocked real-space sum for the bound geometry and the
// current launch shape (two small kernels); once per evaluation, before the
// real-space launches.
void se_launch_real_prep(const se_plan* p, hipStream_t s);
// Work items of the register-tiled gridding and gathering for the bound
// geometry (crowded tiles get items beyond their first); once per evaluation.
void se_launch_tile_prep(const se_plan* p, hipStream_t s);
// Exclusive scan of n ints in place by one workgroup; v[n] receives the total.
void se_launch_scan_excl(int* v, int64_t n, hipStream_t s);
// Direct Ewald reference (se_reference.cpp): all-pairs real space (or the
// free-space sum for D = 0), the explicit k-space lattice sum, and the terms
// outside both (self, stresslet k = 0, harmonic background).
void se_launch_dref_real(int kernel, int D, const double* L, double xi, double rc, int64_t ns, const double* xs,
                         const double* f, const double* nu, int64_t nt, const double* xt, int tas, double* u,
                         int* flags, hipStream_t s);
void se_launch_dref_kspace(int kernel, int nk, const double* kv, double xi, double volume, int64_t ns,
                           const double* xs, const double* f, const double* nu, double* U, int64_t nt,
                           const double* xt, double* u, hipStream_t s);
void se_launch_dref_zero(int kernel, int D, const double* L, double xi, int64_t ns, const double* xs,
                         const double* f, const double* nu, int64_t nt, const double* xt, double* u, hipStream_t s);
void se_launch_dref_terms(int kernel, int D, const double* L, double xi, int64_t ns, const double* xs,
                          const double* f, const double* nu, int64_t nt, const double* xt, int tas, double* sums,
                          double* u, hipStream_t s);
void se_launch_real_space(const se_plan* p, int slot0, int nslot, hipStream_t s);
void se_launch_reductions(const se_plan* p, int slot, hipStream_t s);
void se_fft3d_f64(const int* Mg, const int* N, const double* h, double* grid, double* spec, const double* tw,
                  const int* tw_off, int ncomp, int dir, hipStream_t s);
void se_fft_twiddles(const int* N, std::vector<double>* tw, int* off);
se_status se_d0_precompute(se_plan* p);
bool se_fft_fits(const int* N, int ncomp, bool fp32);
void se_launch_finalize(const se_plan* p, int slot, double* u, double* u_real, double* u_fourier, hipStream_t s);

// Merged launches for batches of systems: one launch of a phase covers the
// work items of many plans.  A job is one plan's share of a phase (one
// right-hand-side slot, or the pair of them that a kernel takes together):
// its kernel family and variant (the template arguments), the workgroups of
// its first-item launch, its dynamic LDS and its argument record.
enum {
    SE_JOB_SPREAD = 0,
    SE_JOB_GATHER = 1,
    SE_JOB_FFT_X_R2C = 2,
    SE_JOB_FFT_Y_FWD = 3,
    SE_JOB_FFT_Z_SCALE = 4,
    SE_JOB_FFT_Y_INV = 5,
    SE_JOB_FFT_X_C2R = 6,
    SE_JOB_REAL = 7,
};
constexpr int SE_JOB_MAX = 1024;  // jobs per merged launch
struct se_job {
    int family = 0;
    int variant = 0;
    int blocks = 0;
    size_t lds = 0;
    std::vector<char> args;
};
// Jobs of one plan for one phase (se_spread.hip, se_fft.hip, se_real.hip);
// false when the plan's phase has no merged form (then it runs alone).
bool se_tile_jobs(const se_plan* p, bool gather, int nslot, std::vector<se_job>* out);
bool se_fft_jobs(const se_plan* p, int family, int slot, std::vector<se_job>* out);
bool se_real_jobs(const se_plan* p, int nslot, std::vector<se_job>* out);
// One merged launch over n jobs of one family and variant: args is the
// device array of their records, boff[0..n] the prefix of their workgroups.
void se_tile_launch_multi(int family, int variant, const void* args, const int* boff, int n, int blocks,
                          hipStream_t s);
void se_fft_launch_multi(int family, int variant, const void* args, const int* boff, int n, int blocks, size_t lds,
                         hipStream_t s);
void se_real_launch_multi(int variant, const void* args, int n, int blocks, hipStream_t s);
int se_real_job_max();  // jobs per merged real-space launch
// The upsampled-class steps of the adaptive FFT (D = 1, 2) of one slot, in
// pipeline order: which = 0 after the x pass, 1 after the y pass, 2 after the
// z pass (class transforms and scaling), 3 after the inverse y pass.
void se_launch_fft_cls(const se_plan* p, int slot, int which, hipStream_t s);

// One evaluation of all right-hand sides of a plan on stream s (kernel
// launches only, so it can be recorded into a graph when timing is off).
extern "C" __attribute__((visibility("hidden"))) se_status se_run_plan(se_plan* p, const double* strengths, double* u,
                                                                        double* ur, double* uf, hipStream_t s);

// Learned-selector kernels (se_mlp.hip).
size_t se_mlp_part_floats(int cnt);
void se_mlp_launch_grad(const float* th, const float* X, const float* Y, int64_t n, uint64_t a, uint64_t c,
                        int64_t start, int cnt, float* part, float* grad, float* loss, hipStream_t s);
void se_mlp_launch_adam(float* th, float* m, float* v, const float* g, int64_t n, int t, float lr, float b1,
                        float b2, float eps, hipStream_t s);
void se_mlp_launch_forward(const float* th, const float* X, int64_t n, float* Y, const float* norm, hipStream_t s);
void se_mlp_launch_fill(float* p, int64_t n, float v, hipStream_t s);
