// se_batch.cpp -- batches of independent systems of uneven size and any
// periodicity, evaluated on one stream and replayed as one HIP graph.
//
// Each member is an ordinary plan (its own parameters from the Sec. 4.6
// procedure, its own grid and cell list).  A batch of several members runs
// phase by phase: one launch per phase covers the work items of all members
// (the tiles of gridding and gathering, the line bundles of every FFT pass,
// the blocks of the real-space sum), reading each member's argument record
// from a device array; only the member-specific steps (strengths, the
// upsampled-class steps of D = 1, 2, the epilogue) are launched per member.
// The batch records this schedule into a graph, and autotunes each member's
// launch shapes (which leave the arithmetic unchanged).
#include "se_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

// Independent systems are recorded on up to kLanes forked streams, so the
// graph holds them as parallel branches and small systems share the chip.
constexpr int kLanes = 4;

// One step of the phase-major schedule: a merged launch over jobs of one
// family and variant, or a step of one member.
struct se_step {
    int kind = 0;  // 0: merged launch, else a member step (below)
    int family = 0, variant = 0, n = 0, blocks = 0;
    size_t lds = 0, args_off = 0, boff_off = 0;
    int plan = 0, r0 = 0, nr = 0, slot = 0, which = 0;
};
enum {
    kStepMerged = 0,
    kStepStrengths,  // strengths, reductions and the cleared Fourier accumulators of a chunk
    kStepPrep,       // per-geometry counts and scans of the tiles and the real-space blocks
    kStepSpread,     // gridding of a member without a merged form
    kStepGather,
    kStepReal,
    kStepCls,        // an upsampled-class step of the adaptive FFT
    kStepFinalize,
};

struct se_batch {
    std::vector<se_plan*> plans;
    // phase-major schedule (batches of two or more members) and its device
    // argument records, rebuilt when a member's launch shapes change
    std::vector<se_step> steps;
    std::vector<uintptr_t> skey;
    char* d_jobs = nullptr;
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;  // stream, pointers and launch shapes the graph holds
    // geometry binding (bin keys, sort, cell starts, sorted copies), recorded
    // the same way and keyed by the stream and the position pointers
    hipGraph_t ggraph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uintptr_t> gkey;
    hipStream_t lane[kLanes] = {};
    hipEvent_t fork = nullptr, join[kLanes] = {};
};

namespace {

void drop_graph(se_batch* b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key.clear();
}

void drop_geometry_graph(se_batch* b)
{
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->ggraph) hipGraphDestroy(b->ggraph);
    b->gexec = nullptr;
    b->ggraph = nullptr;
    b->gkey.clear();
}

// Shapes that the schedule depends on (the merged records hold the plans'
// launch shapes).
std::vector<uintptr_t> schedule_key(const se_batch* b)
{
    std::vector<uintptr_t> k;
    for (const se_plan* p : b->plans) {
        k.push_back((uintptr_t)p->shape_real_tb);
        k.push_back((uintptr_t)p->shape_fft_cols);
        k.push_back((uintptr_t)p->shape_tile_items);
    }
    return k;
}

// Groups jobs by family and variant into merged steps (at most `cap` jobs
// each), appending their records (one struct each, packed as the kernels
// index them) and workgroup prefixes to the host image.
void emit_merged(std::vector<se_job>& jobs, int cap, std::vector<se_step>* steps, std::vector<char>* img)
{
    auto align = [&](size_t a) { img->resize((img->size() + a - 1) / a * a); };
    std::vector<bool> done(jobs.size(), false);
    for (size_t i = 0; i < jobs.size(); i++) {
        if (done[i]) continue;
        std::vector<size_t> grp;
        for (size_t k = i; k < jobs.size(); k++)
            if (!done[k] && jobs[k].family == jobs[i].family && jobs[k].variant == jobs[i].variant) {
                grp.push_back(k);
                done[k] = true;
            }
        for (size_t g0 = 0; g0 < grp.size(); g0 += cap) {
            const size_t g1 = std::min(grp.size(), g0 + cap);
            se_step st;
            st.kind = kStepMerged;
            st.family = jobs[i].family;
            st.variant = jobs[i].variant;
            st.n = (int)(g1 - g0);
            align(256);
            st.args_off = img->size();
            for (size_t k = g0; k < g1; k++) {
                const se_job& j = jobs[grp[k]];
                img->insert(img->end(), j.args.begin(), j.args.end());
                st.lds = std::max(st.lds, j.lds);
            }
            align(256);
            st.boff_off = img->size();
            int acc = 0;
            for (size_t k = g0; k <= g1; k++) {
                const int v = acc;
                img->insert(img->end(), (const char*)&v, (const char*)&v + sizeof(int));
                if (k < g1) acc += jobs[grp[k]].blocks;
            }
            st.blocks = acc;
            steps->push_back(st);
        }
    }
    jobs.clear();
}

// The phase-major schedule of a batch: per chunk of right-hand sides the
// member steps and merged launches in pipeline order.
se_status build_schedule(se_batch* b)
{
    std::vector<se_step> steps;
    std::vector<char> img;
    std::vector<se_job> jobs;
    int nchunk = 0;
    for (const se_plan* p : b->plans) nchunk = std::max(nchunk, (p->nrhs + p->rb - 1) / p->rb);
    auto member = [&](int kind, int i, int r0, int nr, int slot = 0, int which = 0) {
        se_step st;
        st.kind = kind;
        st.plan = i;
        st.r0 = r0;
        st.nr = nr;
        st.slot = slot;
        st.which = which;
        steps.push_back(st);
    };
    const int np = (int)b->plans.size();
    for (int c = 0; c < nchunk; c++) {
        std::vector<int> r0(np), nr(np, 0);
        for (int i = 0; i < np; i++) {
            const se_plan* p = b->plans[i];
            r0[i] = c * p->rb;
            nr[i] = r0[i] < p->nrhs ? std::min(p->rb, p->nrhs - r0[i]) : 0;
        }
        for (int i = 0; i < np; i++)
            if (nr[i]) {
                member(kStepStrengths, i, r0[i], nr[i]);
                if (c == 0) member(kStepPrep, i, 0, nr[i]);
            }
        // gridding
        for (int i = 0; i < np; i++)
            if (nr[i] && !se_tile_jobs(b->plans[i], false, nr[i], &jobs)) member(kStepSpread, i, r0[i], nr[i]);
        emit_merged(jobs, SE_JOB_MAX, &steps, &img);
        // forward transforms: x, class step 0, y, class step 1
        const int fam_fwd[2] = {SE_JOB_FFT_X_R2C, SE_JOB_FFT_Y_FWD};
        for (int pass = 0; pass < 2; pass++) {
            for (int i = 0; i < np; i++)
                for (int k = 0; k < nr[i]; k++) se_fft_jobs(b->plans[i], fam_fwd[pass], k, &jobs);
            emit_merged(jobs, SE_JOB_MAX, &steps, &img);
            for (int i = 0; i < np; i++)
                for (int k = 0; k < nr[i]; k++)
                    if (b->plans[i]->D == 1 || b->plans[i]->D == 2) member(kStepCls, i, r0[i], nr[i], k, pass);
        }
        // z transform, scaling and inverse z; class step 2
        for (int i = 0; i < np; i++)
            for (int k = 0; k < nr[i]; k++) se_fft_jobs(b->plans[i], SE_JOB_FFT_Z_SCALE, k, &jobs);
        emit_merged(jobs, SE_JOB_MAX, &steps, &img);
        for (int i = 0; i < np; i++)
            for (int k = 0; k < nr[i]; k++)
                if (b->plans[i]->D == 1 || b->plans[i]->D == 2) member(kStepCls, i, r0[i], nr[i], k, 2);
        // inverse y, class step 3, inverse x
        for (int i = 0; i < np; i++)
            for (int k = 0; k < nr[i]; k++) se_fft_jobs(b->plans[i], SE_JOB_FFT_Y_INV, k, &jobs);
        emit_merged(jobs, SE_JOB_MAX, &steps, &img);
        for (int i = 0; i < np; i++)
            for (int k = 0; k < nr[i]; k++)
                if (b->plans[i]->D == 1) member(kStepCls, i, r0[i], nr[i], k, 3);
        for (int i = 0; i < np; i++)
            for (int k = 0; k < nr[i]; k++) se_fft_jobs(b->plans[i], SE_JOB_FFT_X_C2R, k, &jobs);
        emit_merged(jobs, SE_JOB_MAX, &steps, &img);
        // gathering
        for (int i = 0; i < np; i++)
            if (nr[i] && !se_tile_jobs(b->plans[i], true, nr[i], &jobs)) member(kStepGather, i, r0[i], nr[i]);
        emit_merged(jobs, SE_JOB_MAX, &steps, &img);
        // real-space sums
        for (int i = 0; i < np; i++)
            if (nr[i] && !se_real_jobs(b->plans[i], nr[i], &jobs)) member(kStepReal, i, r0[i], nr[i]);
        emit_merged(jobs, se_real_job_max(), &steps, &img);
        for (int i = 0; i < np; i++)
            if (nr[i]) member(kStepFinalize, i, r0[i], nr[i]);
    }
    if (b->d_jobs) hipFree(b->d_jobs);
    b->d_jobs = nullptr;
    if (!img.empty()) {
        if (hipMalloc(&b->d_jobs, img.size()) != hipSuccess) return SE_ERR_NOMEM;
        if (hipMemcpy(b->d_jobs, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) return SE_ERR_HIP;
    }
    b->steps = std::move(steps);
    b->skey = schedule_key(b);
    return SE_OK;
}

// One evaluation of every member through the schedule, on stream s.
se_status run_schedule(se_batch* b, const double* const* f, double* const* u, hipStream_t s)
{
    for (const se_step& st : b->steps) {
        se_plan* p = b->plans[st.plan];
        switch (st.kind) {
            case kStepMerged: {
                const void* args = b->d_jobs + st.args_off;
                const int* boff = (const int*)(b->d_jobs + st.boff_off);
                if (st.family == SE_JOB_SPREAD || st.family == SE_JOB_GATHER)
                    se_tile_launch_multi(st.family, st.variant, args, boff, st.n, st.blocks, s);
                else if (st.family == SE_JOB_REAL)
                    se_real_launch_multi(st.variant, args, st.n, st.blocks, s);
                else
                    se_fft_launch_multi(st.family, st.variant, args, boff, st.n, st.blocks, st.lds, s);
                break;
            }
            case kStepStrengths:
                for (int k = 0; k < st.nr; k++) {
                    se_launch_strengths(p, f[st.plan] + (size_t)(st.r0 + k) * p->ns * 3, k, s);
                    se_launch_reductions(p, k, s);
                }
                se_launch_fill_double(p->d_uF, 0.0, (int64_t)st.nr * 3 * p->nt, s);
                break;
            case kStepPrep:
                se_launch_tile_prep(p, s);
                se_launch_real_prep(p, s);
                break;
            case kStepSpread: se_launch_spread(p, 0, st.nr, s); break;
            case kStepGather: se_launch_gather(p, 0, st.nr, s); break;
            case kStepReal: se_launch_real_space(p, 0, st.nr, s); break;
            case kStepCls: se_launch_fft_cls(p, st.slot, st.which, s); break;
            case kStepFinalize:
                for (int k = 0; k < st.nr; k++)
                    se_launch_finalize(p, k, u[st.plan] + (size_t)(st.r0 + k) * p->nt * 3, nullptr, nullptr, s);
                break;
        }
    }
    return hipGetLastError() == hipSuccess ? SE_OK : SE_ERR_HIP;
}

se_status run_eager(se_batch* b, const double* const* f, double* const* u, hipStream_t s)
{
    for (size_t i = 0; i < b->plans.size(); i++) {
        se_status st = se_run_plan(b->plans[i], f[i], u[i], nullptr, nullptr, s);
        if (st != SE_OK) return st;
    }
    return SE_OK;
}

bool make_lanes(se_batch* b)
{
    if (b->fork) return true;
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return false;
    for (int l = 0; l < kLanes; l++) {
        if (hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming) != hipSuccess) return false;
    }
    return true;
}

// Records every member's launches (work(i, stream) for system i) into a
// graph: fork from s onto the lanes, system i on lane i mod kLanes, join back
// on s (timing events off: they would need host synchronisation inside the
// capture).  Every cross-stream dependency goes through s, the stream that
// began the capture.
template <typename Work>
se_status record(se_batch* b, hipStream_t s, Work&& work, hipGraph_t* graph, hipGraphExec_t* exec)
{
    if (!make_lanes(b)) return SE_ERR_HIP;
    std::vector<bool> timing(b->plans.size());
    for (size_t i = 0; i < b->plans.size(); i++) {
        timing[i] = b->plans[i]->timing;
        b->plans[i]->timing = false;
    }
    const int lanes = (int)std::min<size_t>(kLanes, b->plans.size());
    se_status st = SE_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
        st = SE_ERR_HIP;
    } else {
        hipError_t e = hipEventRecord(b->fork, s);
        for (int l = 0; l < lanes && e == hipSuccess; l++) e = hipStreamWaitEvent(b->lane[l], b->fork, 0);
        if (e != hipSuccess) st = SE_ERR_HIP;
        for (size_t i = 0; i < b->plans.size() && st == SE_OK; i++) st = work(i, b->lane[i % lanes]);
        for (int l = 0; l < lanes; l++) {
            hipError_t e1 = hipEventRecord(b->join[l], b->lane[l]);
            if (e1 == hipSuccess) e1 = hipStreamWaitEvent(s, b->join[l], 0);
            if (e1 != hipSuccess && st == SE_OK) st = SE_ERR_HIP;
        }
        e = hipStreamEndCapture(s, &g);
        if (st == SE_OK && (e != hipSuccess || !g)) st = SE_ERR_HIP;
    }
    for (size_t i = 0; i < b->plans.size(); i++) b->plans[i]->timing = timing[i];
    if (st == SE_OK && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
        *exec = nullptr;
        st = SE_ERR_HIP;
    }
    if (st != SE_OK) {
        if (g) hipGraphDestroy(g);
        (void)hipGetLastError();
        return st;
    }
    *graph = g;
    return SE_OK;
}

// Records the schedule on s alone (its only stream) into a graph.
se_status record_schedule(se_batch* b, const double* const* f, double* const* u, hipStream_t s)
{
    se_status st = SE_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return SE_ERR_HIP;
    st = run_schedule(b, f, u, s);
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st == SE_OK && (e != hipSuccess || !g)) st = SE_ERR_HIP;
    if (st == SE_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        st = SE_ERR_HIP;
    }
    if (st != SE_OK) {
        if (g) hipGraphDestroy(g);
        (void)hipGetLastError();
        return st;
    }
    b->graph = g;
    return SE_OK;
}

bool check_args(const se_batch* b, const double* const* f, double* const* u)
{
    if (!b || !f || !u) return false;
    for (size_t i = 0; i < b->plans.size(); i++)
        if (!f[i] || !u[i]) return false;
    return true;
}

}  // namespace

extern "C" {

se_status se_batch_create(const se_problem* probs, int32_t n_sys, se_batch** out)
{
    if (!probs || !out || n_sys <= 0) return SE_ERR_ARG;
    *out = nullptr;
    se_batch* b = new se_batch;
    for (int32_t i = 0; i < n_sys; i++) {
        se_plan* p = nullptr;
        se_status st = se_plan_create(&probs[i], nullptr, &p);
        if (st != SE_OK) {
            for (se_plan* q : b->plans) se_plan_destroy(q);
            delete b;
            return st;
        }
        if (i > 0 && p->device != b->plans[0]->device) {
            se_plan_destroy(p);
            for (se_plan* q : b->plans) se_plan_destroy(q);
            delete b;
            return SE_ERR_ARG;
        }
        b->plans.push_back(p);
    }
    b->device = b->plans[0]->device;
    *out = b;
    return SE_OK;
}

se_status se_batch_destroy(se_batch* b)
{
    if (!b) return SE_ERR_ARG;
    hipSetDevice(b->device);
    hipDeviceSynchronize();
    drop_graph(b);
    drop_geometry_graph(b);
    if (b->d_jobs) hipFree(b->d_jobs);
    if (b->fork) hipEventDestroy(b->fork);
    for (int l = 0; l < kLanes; l++) {
        if (b->lane[l]) hipStreamDestroy(b->lane[l]);
        if (b->join[l]) hipEventDestroy(b->join[l]);
    }
    for (se_plan* p : b->plans) se_plan_destroy(p);
    delete b;
    return SE_OK;
}

se_status se_batch_plan(se_batch* b, int32_t i, se_plan** plan)
{
    if (!b || !plan || i < 0 || i >= (int32_t)b->plans.size()) return SE_ERR_ARG;
    *plan = b->plans[i];
    return SE_OK;
}

se_status se_batch_set_geometry(se_batch* b, const double* const* src, const double* const* nrm,
                                const double* const* tgt, void* stream)
{
    if (!b || !src) return SE_ERR_ARG;
    for (size_t i = 0; i < b->plans.size(); i++)
        if (!src[i]) return SE_ERR_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return SE_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    auto bind = [&](size_t i, hipStream_t st) {
        return se_set_geometry(b->plans[i], src[i], nrm ? nrm[i] : nullptr, tgt ? tgt[i] : nullptr, st);
    };
    // binding rewrites the plans' own cell lists and sorted copies in place,
    // so the evaluation graph stays valid across it; the binding itself is
    // replayed from its own graph while the stream and pointers are unchanged
    std::vector<uintptr_t> key;
    key.push_back((uintptr_t)stream);
    for (size_t i = 0; i < b->plans.size(); i++) {
        key.push_back((uintptr_t)src[i]);
        key.push_back((uintptr_t)(nrm ? nrm[i] : nullptr));
        key.push_back((uintptr_t)(tgt ? tgt[i] : nullptr));
    }
    bool bound = true;
    for (se_plan* p : b->plans) bound = bound && p->have_geometry;
    if (s && b->gexec && bound && key == b->gkey) return hipGraphLaunch(b->gexec, s) == hipSuccess ? SE_OK : SE_ERR_HIP;
    drop_geometry_graph(b);
    for (size_t i = 0; i < b->plans.size(); i++) {
        se_status st = bind(i, s);
        if (st != SE_OK) return st;
    }
    // the eager pass above is the result of this call; the graph serves the next ones
    if (s && record(b, s, bind, &b->ggraph, &b->gexec) == SE_OK) b->gkey = key;
    return SE_OK;
}

se_status se_batch_execute(se_batch* b, const double* const* f, double* const* u, void* stream)
{
    if (!check_args(b, f, u)) return SE_ERR_ARG;
    for (se_plan* p : b->plans)
        if (!p->have_geometry) return SE_ERR_STATE;
    if (hipSetDevice(b->device) != hipSuccess) return SE_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    // several members: the phase-major schedule (merged launches)
    const bool merged = b->plans.size() >= 2;
    if (merged && (b->steps.empty() || b->skey != schedule_key(b))) {
        drop_graph(b);
        se_status st = build_schedule(b);
        if (st != SE_OK) return st;
    }
    if (!s) return merged ? run_schedule(b, f, u, s) : run_eager(b, f, u, s);

    std::vector<uintptr_t> key;
    key.reserve(5 * b->plans.size() + 1);
    key.push_back((uintptr_t)stream);
    for (size_t i = 0; i < b->plans.size(); i++) {
        const se_plan* p = b->plans[i];
        key.push_back((uintptr_t)f[i]);
        key.push_back((uintptr_t)u[i]);
        key.push_back((uintptr_t)p->shape_real_tb);
        key.push_back((uintptr_t)p->shape_fft_cols);
        key.push_back((uintptr_t)p->shape_tile_items);
    }
    if (b->exec && key == b->key) return hipGraphLaunch(b->exec, s) == hipSuccess ? SE_OK : SE_ERR_HIP;

    drop_graph(b);
    se_status st = merged ? run_schedule(b, f, u, s) : run_eager(b, f, u, s);
    if (st != SE_OK) return st;
    // the eager pass above is the result of this call; the graph serves the next ones
    if (merged) {
        if (record_schedule(b, f, u, s) == SE_OK) b->key = key;
    } else {
        auto run = [&](size_t i, hipStream_t st) { return se_run_plan(b->plans[i], f[i], u[i], nullptr, nullptr, st); };
        if (record(b, s, run, &b->graph, &b->exec) == SE_OK) b->key = key;
    }
    return SE_OK;
}

se_status se_batch_tune(se_batch* b, const double* const* f, double* const* u, void* stream)
{
    if (!check_args(b, f, u)) return SE_ERR_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return SE_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    drop_graph(b);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return SE_ERR_HIP;
    }
    se_status st = SE_OK;
    for (size_t i = 0; i < b->plans.size() && st == SE_OK; i++) {
        se_plan* p = b->plans[i];
        if (!p->have_geometry) {
            st = SE_ERR_STATE;
            break;
        }
        const bool timing = p->timing;
        p->timing = false;
        // the knobs act on different phases: tune one after the other
        const int tbs[5] = {0, 1, 2, 3, 4};
        const int cols[5] = {0, 2, 4, 8, 16};
        const int items[5] = {0, 4, 8, 16, 64};
        int best_tb = 0, best_cols = 0, best_items = 0;
        for (int pass = 0; pass < 3 && st == SE_OK; pass++) {
            float best = 1e30f;
            for (int c = 0; c < 5; c++) {
                const int tb = pass == 0 ? tbs[c] : best_tb;
                const int fc = pass == 0 ? 0 : (pass == 1 ? cols[c] : best_cols);
                const int ti = pass == 2 ? items[c] : 0;
                p->shape_real_tb = tb;
                p->shape_fft_cols = fc;
                p->shape_tile_items = ti;
                st = se_run_plan(p, f[i], u[i], nullptr, nullptr, s);  // warm-up
                if (st != SE_OK) break;
                float ms = 0.f;
                hipEventRecord(e0, s);
                for (int r = 0; r < 2 && st == SE_OK; r++) st = se_run_plan(p, f[i], u[i], nullptr, nullptr, s);
                hipEventRecord(e1, s);
                if (st != SE_OK || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    if (st == SE_OK) st = SE_ERR_HIP;
                    break;
                }
                if (ms < best) {
                    best = ms;
                    if (pass == 0) best_tb = tb;
                    else if (pass == 1) best_cols = fc;
                    else best_items = ti;
                }
            }
        }
        p->shape_real_tb = best_tb;
        p->shape_fft_cols = best_cols;
        p->shape_tile_items = best_items;
        p->timing = timing;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return st;
}

}  // extern "C"
