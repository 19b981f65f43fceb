// se_batch.cpp -- batches of independent systems of uneven size and any
// periodicity, evaluated on one stream and replayed as one HIP graph.
//
// Each member is an ordinary plan (its own parameters from the Sec. 4.6
// procedure, its own grid and cell list); the batch adds the launch-level
// plumbing: a graph that holds every member's full evaluation (strengths
// through finalisation, Secs. 3.2-3.3 and 4), and a per-member autotuner over
// the launch shapes that leave the arithmetic unchanged.
#include "se_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

// Independent systems are recorded on up to kLanes forked streams, so the
// graph holds them as parallel branches and small systems share the chip.
constexpr int kLanes = 4;

struct se_batch {
    std::vector<se_plan*> plans;
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
    if (!s) return run_eager(b, f, u, s);

    std::vector<uintptr_t> key;
    key.reserve(4 * b->plans.size() + 1);
    key.push_back((uintptr_t)stream);
    for (size_t i = 0; i < b->plans.size(); i++) {
        const se_plan* p = b->plans[i];
        key.push_back((uintptr_t)f[i]);
        key.push_back((uintptr_t)u[i]);
        key.push_back((uintptr_t)p->shape_real_tb);
        key.push_back((uintptr_t)p->shape_fft_cols);
    }
    if (b->exec && key == b->key) return hipGraphLaunch(b->exec, s) == hipSuccess ? SE_OK : SE_ERR_HIP;

    drop_graph(b);
    se_status st = run_eager(b, f, u, s);
    if (st != SE_OK) return st;
    // the eager pass above is the result of this call; the graph serves the next ones
    auto run = [&](size_t i, hipStream_t st) { return se_run_plan(b->plans[i], f[i], u[i], nullptr, nullptr, st); };
    if (record(b, s, run, &b->graph, &b->exec) == SE_OK) b->key = key;
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
        // the two knobs act on different phases: tune one, then the other
        const int tbs[5] = {0, 1, 2, 3, 4};
        const int cols[5] = {0, 2, 4, 8, 16};
        int best_tb = 0, best_cols = 0;
        for (int pass = 0; pass < 2 && st == SE_OK; pass++) {
            float best = 1e30f;
            for (int c = 0; c < 5; c++) {
                const int tb = pass == 0 ? tbs[c] : best_tb;
                const int fc = pass == 0 ? 0 : cols[c];
                p->shape_real_tb = tb;
                p->shape_fft_cols = fc;
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
                    else best_cols = fc;
                }
            }
        }
        p->shape_real_tb = best_tb;
        p->shape_fft_cols = best_cols;
        p->timing = timing;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return st;
}

}  // extern "C"
