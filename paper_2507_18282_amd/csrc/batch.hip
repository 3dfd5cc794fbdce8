// ew_batch: many independent Dirichlet rectangles (explicit leapfrog, FP32 or
// FP64 state and filter accumulation, FP64 vectors and Arnoldi) advanced
// together.
//
// One batched wave-solve is a captured hipGraph: with FP32 state the small
// problems run their whole wave-solve in one LDS-resident workgroup each
// (k_batch_small, on a forked branch), while every large problem advances one
// time step per k_batch_step launch (one launch per step index, blocks of
// problems that are already done exit at once); the tile height of
// k_batch_step is chosen at creation by timing the candidates on the batch
// itself.  With FP64 state every problem advances 8 / R steps per
// k_batch_blocked launch (R the stencil's radius), reading the caller's v as
// W^0 and accumulating straight into the caller's out.  The Arnoldi process
// of every problem advances in lock-step: one batched wave-solve, then one
// batched chain of modified Gram-Schmidt links, then the small host-side
// Krylov-Schur bookkeeping of each problem.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "batch.h"
#include "eigs_core.h"
#include "op.h"

namespace ew {

struct BProb {
    Geo g{};
    int64_t N = 0;
    double h[3] = {1, 1, 1};
    TimePlan tp;
    bool small = false;
    void* f0 = nullptr;  // FP32 state only (FP64 state reads v and writes out)
    void* fA = nullptr;
    void* fB = nullptr;
    void* fC = nullptr;  // FP64 state only: the second pair of time levels
    void* fD = nullptr;
    void* acc = nullptr;
};

}  // namespace ew

struct ew_batch_s {
    int nprob = 0;
    int order = 2;
    int fp64 = 0;  // state type: FP64 (precision EW_PREC_FP64) or FP32 (EW_PREC_MIXED)
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;  // private stream the graph runs on
    hipStream_t side = nullptr;    // branch for the small problems
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_in = nullptr, ev_out = nullptr, ev_copy = nullptr;
    std::vector<ew::BProb> P;
    ew::BatchProbDev* probs_dev = nullptr;
    ew::BatchProbDev* probs_host = nullptr;  // pinned
    void* coef_dev = nullptr;  // filter weights in the state type
    std::vector<int> small_ids, large_ids;
    int* small_ids_dev = nullptr;
    int* large_ids_dev = nullptr;
    ew::BatchBlk* step_tab_dev = nullptr;  // (problem, tile) per step workgroup, sized for the shortest tiles
    int* conv_blk_dev = nullptr;
    int nblocks_step = 0, nblocks_conv = 0, max_nt_large = 0, tyr = 4;
    // Large problems are ordered by N_t, longest first, so the problems that
    // still step at step index s are a prefix: step_nblk[s] blocks cover them.
    std::vector<int> step_nblk;
    // FP64 state: several steps per launch in 16 x 16 tiles, problems in the
    // same order; blk_nblk[L] blocks cover the problems stepping in launch L
    ew::BatchBlk* blk_tab_dev = nullptr;
    std::vector<int> blk_nblk;
    int steps_per_launch = 1;
    size_t small_lds = 0;
    double tune_us[4] = {0, 0, 0, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> allocs;
    int64_t wave_solves = 0, pt_updates = 0;
    ~ew_batch_s();
};

namespace ew {

static ew_status balloc(ew_batch b, void** p, size_t bytes) {
    hipError_t e = dev_alloc(p, bytes, b->user_stream);
    if (e != hipSuccess) return fail(EW_ERR_OOM, std::string("batch allocation: ") + hipGetErrorString(e));
    b->allocs.push_back(*p);
    return EW_OK;
}

static int step_tiles(const Geo& g, int tyr) { return ((g.nx + 63) / 64) * ((g.ny + 4 * tyr - 1) / (4 * tyr)); }

static ew_status build_step_table(ew_batch b, int tyr) {
    std::vector<int> starts(b->large_ids.size() + 1, 0);
    for (size_t s = 0; s < b->large_ids.size(); ++s)
        starts[s + 1] = starts[s] + step_tiles(b->P[b->large_ids[s]].g, tyr);
    b->nblocks_step = starts.back();
    std::vector<BatchBlk> tab(b->nblocks_step);
    for (size_t s = 0; s < b->large_ids.size(); ++s)
        for (int t = starts[s]; t < starts[s + 1]; ++t) tab[t] = {b->large_ids[s], t - starts[s]};
    b->step_nblk.assign(b->max_nt_large, 0);
    size_t cnt = b->large_ids.size();
    for (int st = 0; st < b->max_nt_large; ++st) {  // cnt: problems with N_t > st
        while (cnt > 0 && b->P[b->large_ids[cnt - 1]].tp.n_t <= st) --cnt;
        b->step_nblk[st] = starts[cnt];
    }
    if (!tab.empty())
        EW_HIP_TRY(hipMemcpy(b->step_tab_dev, tab.data(), tab.size() * sizeof(BatchBlk), hipMemcpyHostToDevice));
    b->tyr = tyr;
    return EW_OK;
}

// FP64 state: (problem, tile) of every k_batch_blocked workgroup, the
// problems in the order of large_ids (longest N_t first), and the blocks that
// cover the problems still stepping in each launch.
static ew_status build_blocked_table(ew_batch b) {
    b->steps_per_launch = batch_steps_per_launch(b->order);
    const int spl = b->steps_per_launch;
    std::vector<int> starts(b->large_ids.size() + 1, 0);
    for (size_t s = 0; s < b->large_ids.size(); ++s)
        starts[s + 1] = starts[s] + batch_blocked_tiles(b->P[b->large_ids[s]].g);
    std::vector<BatchBlk> tab(starts.back());
    for (size_t s = 0; s < b->large_ids.size(); ++s)
        for (int t = starts[s]; t < starts[s + 1]; ++t) tab[t] = {b->large_ids[s], t - starts[s]};
    const int nlaunch = (b->max_nt_large + spl - 1) / spl;
    b->blk_nblk.assign(nlaunch, 0);
    size_t cnt = b->large_ids.size();
    for (int l = 0; l < nlaunch; ++l) {  // cnt: problems with N_t > l spl
        while (cnt > 0 && b->P[b->large_ids[cnt - 1]].tp.n_t <= l * spl) --cnt;
        b->blk_nblk[l] = starts[cnt];
    }
    EW_TRY(balloc(b, (void**)&b->blk_tab_dev, (tab.size() + 1) * sizeof(BatchBlk)));
    if (!tab.empty())
        EW_HIP_TRY(hipMemcpy(b->blk_tab_dev, tab.data(), tab.size() * sizeof(BatchBlk), hipMemcpyHostToDevice));
    return EW_OK;
}

// One batched wave-solve as a graph on b->stream.
static ew_status capture_graph(ew_batch b) {
    hipStream_t s = b->stream;
    EW_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    const int nl = (int)b->large_ids.size(), ns = (int)b->small_ids.size();
    if (nl > 0 && !b->fp64)
        e = launch_batch_convert(b->probs_dev, b->large_ids_dev, b->conv_blk_dev, nl, b->nblocks_conv, 1, s);
    if (e == hipSuccess && ns > 0) {
        e = hipEventRecord(b->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
        if (e == hipSuccess)
            e = launch_batch_small(b->probs_dev, b->small_ids_dev, ns, static_cast<const float*>(b->coef_dev), b->order,
                                   b->small_lds, b->side);
        if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->side);
    }
    if (b->fp64) {
        for (int l = 0; e == hipSuccess && l < (int)b->blk_nblk.size(); ++l)
            e = launch_batch_blocked(b->probs_dev, b->blk_tab_dev, b->blk_nblk[l],
                                     static_cast<const double*>(b->coef_dev), l, b->order, s);
    } else {
        for (int step = 0; e == hipSuccess && step < b->max_nt_large; ++step)
            e = launch_batch_step(b->probs_dev, b->step_tab_dev, b->step_nblk[step], b->coef_dev, step, b->order,
                                  b->tyr, b->fp64, s);
    }
    if (e == hipSuccess && nl > 0 && !b->fp64)
        e = launch_batch_convert(b->probs_dev, b->large_ids_dev, b->conv_blk_dev, nl, b->nblocks_conv, 0, s);
    if (e == hipSuccess && ns > 0) e = hipStreamWaitEvent(s, b->ev_join, 0);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return fail(EW_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(EW_ERR_HIP, std::string("batch graph end capture: ") + hipGetErrorString(e2));
    b->graph = g;
    EW_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return EW_OK;
}

// Time k_batch_step for every tile height on the batch itself (step index 1
// on the zero-initialised FP32 buffers) and keep the fastest.  FP64 state
// runs k_batch_blocked, which has no such choice.
static ew_status autotune(ew_batch b) {
    if (b->large_ids.empty() || b->fp64) return EW_OK;
    for (int i = 0; i < b->nprob; ++i) {
        b->probs_host[i].active = b->P[i].small ? 0 : 1;
        b->probs_host[i].v = nullptr;
        b->probs_host[i].out = nullptr;
    }
    EW_HIP_TRY(hipMemcpy(b->probs_dev, b->probs_host, b->nprob * sizeof(BatchProbDev), hipMemcpyHostToDevice));
    const int cand[4] = {1, 2, 4, 8};
    hipEvent_t e0, e1;
    EW_HIP_TRY(hipEventCreate(&e0));
    EW_HIP_TRY(hipEventCreate(&e1));
    double best = 1e30;
    int best_tyr = 4;
    for (int c = 0; c < 4; ++c) {
        EW_TRY(build_step_table(b, cand[c]));
        EW_HIP_TRY(launch_batch_step(b->probs_dev, b->step_tab_dev, b->nblocks_step, b->coef_dev, 1, b->order, cand[c],
                                     b->fp64, b->stream));
        EW_HIP_TRY(hipEventRecord(e0, b->stream));
        for (int r = 0; r < 8; ++r)
            EW_HIP_TRY(launch_batch_step(b->probs_dev, b->step_tab_dev, b->nblocks_step, b->coef_dev, 1, b->order,
                                         cand[c], b->fp64, b->stream));
        EW_HIP_TRY(hipEventRecord(e1, b->stream));
        EW_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        EW_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        b->tune_us[c] = ms * 1e3 / 8.0;
        if (b->tune_us[c] < best) {
            best = b->tune_us[c];
            best_tyr = cand[c];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    EW_HIP_TRY(hipStreamSynchronize(b->stream));
    return build_step_table(b, best_tyr);
}

// One batched wave-solve out[i] = S_i v[i] for the problems with active[i].
static ew_status batch_apply(ew_batch b, const double* const* v, double* const* out, const char* active) {
    EW_HIP_TRY(hipEventSynchronize(b->ev_copy));  // the previous table upload has finished
    for (int i = 0; i < b->nprob; ++i) {
        b->probs_host[i].v = v[i];
        b->probs_host[i].out = out[i];
        b->probs_host[i].active = active ? (active[i] ? 1 : 0) : 1;
        if (b->fp64) {
            b->probs_host[i].f0 = const_cast<double*>(v[i]);
            b->probs_host[i].acc = out[i];
        }
    }
    EW_HIP_TRY(hipEventRecord(b->ev_in, b->user_stream));
    EW_HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    EW_HIP_TRY(hipMemcpyAsync(b->probs_dev, b->probs_host, b->nprob * sizeof(BatchProbDev), hipMemcpyHostToDevice,
                              b->stream));
    EW_HIP_TRY(hipEventRecord(b->ev_copy, b->stream));
    EW_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    EW_HIP_TRY(hipEventRecord(b->ev_out, b->stream));
    EW_HIP_TRY(hipStreamWaitEvent(b->user_stream, b->ev_out, 0));
    for (int i = 0; i < b->nprob; ++i) {
        if (active && !active[i]) continue;
        b->wave_solves++;
        b->pt_updates += b->P[i].N * (int64_t)b->P[i].tp.n_t;
    }
    return EW_OK;
}

}  // namespace ew

ew_batch_s::~ew_batch_s() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    for (void* p : allocs) ew::dev_free(p);
    if (probs_host) hipHostFree(probs_host);
    for (hipEvent_t e : {ev_fork, ev_join, ev_in, ev_out, ev_copy})
        if (e) hipEventDestroy(e);
    if (side) hipStreamDestroy(side);
    if (stream) hipStreamDestroy(stream);
}

using namespace ew;

extern "C" ew_status ew_batch_create(int nprob, const ew_grid_desc* grids, const ew_op_desc* descs, void* hip_stream,
                                     ew_batch* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (nprob < 1 || nprob > 65536 || !grids || !descs) return fail(EW_ERR_INVALID_ARG, "need 1 <= nprob <= 65536");
    std::unique_ptr<ew_batch_s> b(new ew_batch_s());
    b->nprob = nprob;
    b->order = grids[0].order;
    b->user_stream = (hipStream_t)hip_stream;
    b->P.resize(nprob);
    b->fp64 = descs[0].precision == EW_PREC_FP64 ? 1 : 0;
    std::vector<double> coef;
    std::vector<int> coef_off(nprob);
    for (int i = 0; i < nprob; ++i) {
        EW_TRY(validate_descs(&grids[i], &descs[i]));
        if (grids[i].dim != 2) return fail(EW_ERR_UNSUPPORTED, "the batched form takes 2D problems");
        for (int d = 0; d < 2; ++d)
            if (grids[i].walls[d][0] != EW_WALL_DIRICHLET || grids[i].walls[d][1] != EW_WALL_DIRICHLET)
                return fail(EW_ERR_UNSUPPORTED, "the batched form takes Dirichlet rectangles");
        if (descs[i].ts != EW_TS_EXPLICIT) return fail(EW_ERR_UNSUPPORTED, "the batched form uses explicit stepping");
        if (descs[i].precision != EW_PREC_MIXED && descs[i].precision != EW_PREC_FP64)
            return fail(EW_ERR_UNSUPPORTED, "the batched form keeps FP32 (EW_PREC_MIXED) or FP64 state");
        if ((descs[i].precision == EW_PREC_FP64) != (b->fp64 != 0))
            return fail(EW_ERR_INVALID_ARG, "all problems of a batch share one precision");
        if (grids[i].order != b->order) return fail(EW_ERR_INVALID_ARG, "all problems of a batch share one order");
        BProb& p = b->P[i];
        for (int k = 0; k < 2; ++k) p.h[k] = grids[i].len[k] / (double)(grids[i].n[k] + 1);
        p.g = make_geo(2, grids[i].n, p.h);
        p.N = p.g.size();
        make_time_plan(2, b->order, p.h, descs[i], p.tp);
        p.small = !b->fp64 && p.g.nx <= kBatchSmallMaxSide && p.g.ny <= kBatchSmallMaxSide;
        coef_off[i] = (int)coef.size();
        for (double c : p.tp.c) coef.push_back(c);
    }
    EW_HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    EW_HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    EW_HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    EW_HIP_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    EW_HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    EW_HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    EW_HIP_TRY(hipEventCreateWithFlags(&b->ev_copy, hipEventDisableTiming));
    EW_HIP_TRY(hipEventRecord(b->ev_copy, b->stream));
    if (b->fp64) {
        EW_TRY(balloc(b.get(), &b->coef_dev, coef.size() * sizeof(double)));
        EW_HIP_TRY(hipMemcpy(b->coef_dev, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        const std::vector<float> cf(coef.begin(), coef.end());
        EW_TRY(balloc(b.get(), &b->coef_dev, cf.size() * sizeof(float)));
        EW_HIP_TRY(hipMemcpy(b->coef_dev, cf.data(), cf.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    EW_HIP_TRY(hipHostMalloc((void**)&b->probs_host, nprob * sizeof(BatchProbDev), hipHostMallocDefault));
    EW_TRY(balloc(b.get(), (void**)&b->probs_dev, nprob * sizeof(BatchProbDev)));
    std::vector<int> conv_starts(1, 0);
    for (int i = 0; i < nprob; ++i) {
        BProb& p = b->P[i];
        BatchProbDev& d = b->probs_host[i];
        std::memset(&d, 0, sizeof(d));
        d.g = p.g;
        d.order = b->order;
        d.n_t = p.tp.n_t;
        d.dt2 = b->fp64 ? p.tp.dt * p.tp.dt : (double)(float)(p.tp.dt * p.tp.dt);
        d.coef_off = coef_off[i];
        if (p.small) {
            b->small_ids.push_back(i);
            b->small_lds = std::max(b->small_lds, (size_t)(p.g.nx + 4) * (p.g.ny + 4) * sizeof(float));
        } else {
            b->large_ids.push_back(i);
            b->max_nt_large = std::max(b->max_nt_large, p.tp.n_t);
            if (b->fp64) {
                for (void** z : {&p.fA, &p.fB, &p.fC, &p.fD}) EW_TRY(balloc(b.get(), z, p.N * sizeof(double)));
            } else {
                for (void** z : {&p.f0, &p.fA, &p.fB, &p.acc}) {
                    EW_TRY(balloc(b.get(), z, p.N * sizeof(float)));
                    EW_HIP_TRY(launch_fill<float>(static_cast<float*>(*z), p.N, 0.0f, b->stream));
                }
            }
            d.f0 = p.f0;
            d.fA = p.fA;
            d.fB = p.fB;
            d.fC = p.fC;
            d.fD = p.fD;
            d.acc = p.acc;
        }
    }
    std::stable_sort(b->large_ids.begin(), b->large_ids.end(),
                     [&](int x, int y) { return b->P[x].tp.n_t > b->P[y].tp.n_t; });
    for (int i : b->large_ids)
        conv_starts.push_back(conv_starts.back() +
                              (int)((b->P[i].N + 256 * kConvPerThread - 1) / (256 * kConvPerThread)));
    b->nblocks_conv = conv_starts.back();
    EW_TRY(balloc(b.get(), (void**)&b->small_ids_dev, (b->small_ids.size() + 1) * sizeof(int)));
    EW_TRY(balloc(b.get(), (void**)&b->large_ids_dev, (b->large_ids.size() + 1) * sizeof(int)));
    size_t max_step_blocks = 1;  // the table for the shortest tiles (one row per thread) is the largest
    for (int i : b->large_ids) max_step_blocks += step_tiles(b->P[i].g, 1);
    EW_TRY(balloc(b.get(), (void**)&b->step_tab_dev, max_step_blocks * sizeof(BatchBlk)));
    EW_TRY(balloc(b.get(), (void**)&b->conv_blk_dev, conv_starts.size() * sizeof(int)));
    if (!b->small_ids.empty())
        EW_HIP_TRY(hipMemcpy(b->small_ids_dev, b->small_ids.data(), b->small_ids.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!b->large_ids.empty())
        EW_HIP_TRY(hipMemcpy(b->large_ids_dev, b->large_ids.data(), b->large_ids.size() * sizeof(int), hipMemcpyHostToDevice));
    EW_HIP_TRY(hipMemcpy(b->conv_blk_dev, conv_starts.data(), conv_starts.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!b->small_ids.empty()) EW_HIP_TRY(prepare_batch_small(b->order, b->small_lds));
    if (b->fp64) EW_TRY(build_blocked_table(b.get()));
    EW_HIP_TRY(hipStreamSynchronize(b->stream));
    EW_TRY(autotune(b.get()));
    EW_TRY(capture_graph(b.get()));
    *out = b.release();
    return EW_OK;
}

extern "C" void ew_batch_destroy(ew_batch b) { delete b; }

extern "C" ew_status ew_batch_get_info(ew_batch b, ew_batch_info* out) {
    if (!b || !out) return fail(EW_ERR_INVALID_ARG, "null argument");
    out->nprob = b->nprob;
    out->n_small = (int)b->small_ids.size();
    out->n_large = (int)b->large_ids.size();
    out->max_steps_large = b->max_nt_large;
    out->step_rows_per_thread = b->fp64 ? 0 : b->tyr;
    for (int c = 0; c < 4; ++c) out->tune_us[c] = b->tune_us[c];
    int64_t steps = 0, pts = 0;
    for (const BProb& p : b->P) {
        steps += p.tp.n_t;
        pts += p.N * (int64_t)p.tp.n_t;
    }
    out->total_steps = steps;
    out->pt_updates_per_wave_solve = pts;
    out->state_fp64 = b->fp64;
    out->steps_per_launch = b->fp64 ? b->steps_per_launch : 1;
    return EW_OK;
}

extern "C" ew_status ew_batch_n_active(ew_batch b, int i, int64_t* n_active, int* n_t) {
    if (!b || i < 0 || i >= b->nprob) return fail(EW_ERR_INVALID_ARG, "bad problem index");
    if (n_active) *n_active = b->P[i].N;
    if (n_t) *n_t = b->P[i].tp.n_t;
    return EW_OK;
}

extern "C" ew_status ew_batch_apply_filter(ew_batch b, const double* const* v_dev, double* const* out_dev) {
    if (!b || !v_dev || !out_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < b->nprob; ++i)
        if (!v_dev[i] || !out_dev[i] || v_dev[i] == out_dev[i]) return fail(EW_ERR_INVALID_ARG, "bad vector pointer");
    return batch_apply(b, v_dev, out_dev, nullptr);
}

// ---------------------------------------------------------------------------
// Batched eigensolver
// ---------------------------------------------------------------------------
namespace ew {
namespace {

struct BEig {
    Workspace ws;
    int k = 0, m = 0, n_keep = 0, max_probes = 16;
    double tol_ritz = 1e-12, tol_res = 1e-8;
    int64_t max_ws = 0;
    uint64_t seed = 0;
    const double* v0 = nullptr;
    int phase = 0;  // 0: start a run, 1: Arnoldi steps, 2: done
    int probe = 0, runs = 0, nl = 0, p = 0, j = 0;
    Mat T;
    std::vector<double> th_locked;
    double floor_abs = 0.0;
    int64_t wave_solves = 0, restarts = 0, pt_updates = 0;
    bool budget_hit = false;
    ew_status status = EW_OK;
};

// Ritz analysis at the end of a cycle (same rule as the single-problem run).
// Returns true when the run ends; otherwise the basis has been restarted.
ew_status end_of_cycle(BEig& e, bool& run_ended, std::vector<double>& theta, Mat& Q, std::vector<char>& conv) {
    const int m = e.m;
    Mat A(m, m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A(i, j) = 0.5 * (e.T(i, j) + e.T(j, i));
    std::vector<double> w0;
    Mat Q0;
    sym_eigh(A, w0, Q0);
    std::vector<int> idx = order_by_abs_desc(w0);
    theta.assign(m, 0.0);
    Q = Mat(m, m);
    for (int c = 0; c < m; ++c) {
        theta[c] = w0[idx[c]];
        for (int i = 0; i < m; ++i) Q(i, c) = Q0(i, idx[c]);
    }
    const double beta_m = e.T(m, m - 1);
    conv.assign(m, 0);
    for (int c = 0; c < m; ++c) conv[c] = std::fabs(beta_m * Q(m - 1, c)) <= e.tol_ritz * std::fabs(theta[c]);
    const int nlead = leading_converged(conv);
    bool stop = false;
    if (e.probe == 0) {
        stop = nlead >= e.k;
    } else if (conv[0]) {
        if (std::fabs(theta[0]) < e.floor_abs) stop = true;
        else {
            int n_band = 0;
            for (int c = 0; c < m; ++c) n_band += std::fabs(theta[c]) >= e.floor_abs;
            stop = nlead >= n_band;
        }
    }
    if (stop || e.wave_solves >= e.max_ws) {
        run_ended = true;
        return EW_OK;
    }
    run_ended = false;
    EW_TRY(rotate(e.ws, e.ws.V, m, Q, e.n_keep, e.ws.Vt));
    EW_HIP_TRY(hipMemcpyAsync(e.ws.col(e.ws.Vt, e.n_keep), e.ws.col(e.ws.V, m), e.ws.N * sizeof(double),
                              hipMemcpyDeviceToDevice, e.ws.stream));
    std::swap(e.ws.V, e.ws.Vt);
    e.T = Mat(m + 1, m);
    for (int c = 0; c < e.n_keep; ++c) {
        e.T(c, c) = theta[c];
        e.T(e.n_keep, c) = beta_m * Q(m - 1, c);
    }
    e.p = e.j = e.n_keep;
    e.restarts++;
    return EW_OK;
}

// Lock the converged pairs of a finished run and decide what comes next
// (same rule as the single-problem driver).
ew_status finish_run(BEig& e, const std::vector<double>& theta, const Mat& Q, const std::vector<char>& conv) {
    const int m = e.m;
    if (e.wave_solves >= e.max_ws) e.budget_hit = true;
    int nlead = leading_converged(conv);
    if (e.probe == 0 && nlead < e.k) {
        e.phase = 2;
        return EW_OK;
    }
    if (e.probe > 0) {
        if (!conv[0] || std::fabs(theta[0]) < e.floor_abs) {
            if (conv[0]) e.budget_hit = false;
            e.phase = 2;
            return EW_OK;
        }
        int n_band = 0;
        for (int c = 0; c < m; ++c) n_band += std::fabs(theta[c]) >= e.floor_abs;
        nlead = std::min(nlead, n_band);
    }
    nlead = std::min(nlead, e.ws.cap_lock - e.nl);
    if (nlead <= 0) {
        e.phase = 2;
        return EW_OK;
    }
    EW_TRY(rotate(e.ws, e.ws.V, m, Q, nlead, e.ws.col(e.ws.Y, e.nl)));
    for (int c = 0; c < nlead; ++c) e.th_locked.push_back(theta[c]);
    e.nl += nlead;
    if (e.budget_hit || e.nl >= e.ws.cap_lock) {
        e.phase = 2;
        return EW_OK;
    }
    e.probe++;
    e.phase = (e.probe >= e.max_probes) ? 2 : 0;
    return EW_OK;
}

ew_status start_run(BEig& e) {
    if (e.probe == 0 && e.v0) {
        EW_HIP_TRY(hipMemcpyAsync(e.ws.V, e.v0, e.ws.N * sizeof(double), hipMemcpyDeviceToDevice, e.ws.stream));
    } else {
        EW_HIP_TRY(launch_splitmix_uniform(e.ws.V, e.ws.N, e.seed + (uint64_t)e.probe, e.ws.stream));
    }
    if (e.probe > 0) {
        std::vector<double> a(e.th_locked.size());
        for (size_t i = 0; i < a.size(); ++i) a[i] = std::fabs(e.th_locked[i]);
        std::sort(a.begin(), a.end(), std::greater<double>());
        e.floor_abs = (1.0 - 1e-10) * a[e.k - 1];
    }
    std::vector<const double*> u;
    for (int i = 0; i < e.nl; ++i) u.push_back(e.ws.col(e.ws.Y, i));
    std::vector<double> coeff;
    EW_TRY(mgs_orthonormalize(e.ws, e.ws.V, u, coeff));
    if (!(coeff.back() > 0.0)) return fail(EW_ERR_NONFINITE, "start vector lies in the locked space");
    e.T = Mat(e.m + 1, e.m);
    e.p = e.j = 0;
    e.phase = 1;
    e.runs++;
    return EW_OK;
}

}  // namespace
}  // namespace ew

extern "C" ew_status ew_batch_eigs(ew_batch b, const ew_eigs_desc* descs, int k_cap, double* mu_host,
                                   double* beta_host, double* res_host, int* n_conv_host, double* const* Y_dev,
                                   ew_eigs_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!b || !descs) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (k_cap < 0 || (k_cap > 0 && (!mu_host || !beta_host || !res_host)))
        return fail(EW_ERR_INVALID_ARG, "k_cap > 0 needs mu_host, beta_host and res_host");
    const int np = b->nprob;
    std::vector<std::unique_ptr<BEig>> E(np);
    for (int i = 0; i < np; ++i) {
        const ew_eigs_desc& d = descs[i];
        const int64_t N = b->P[i].N;
        if (d.k < 1 || d.m <= d.k || d.m > 256 || (int64_t)d.m > N)
            return fail(EW_ERR_INVALID_ARG, "need 1 <= k < m <= min(256, n_active) for every problem");
        if (!(d.tol_ritz > 0.0) || !(d.tol_res > 0.0) || d.max_wave_solves < 1)
            return fail(EW_ERR_INVALID_ARG, "bad tolerances or budget");
        E[i].reset(new BEig());
        BEig& e = *E[i];
        e.k = d.k;
        e.m = d.m;
        e.n_keep = std::min(d.n_keep > 0 ? d.n_keep : std::max(d.k, (d.m + d.k) / 2), d.m - 1);
        if (e.n_keep < e.k) return fail(EW_ERR_INVALID_ARG, "n_keep must be >= k");
        e.max_probes = d.max_probes > 0 ? d.max_probes : 16;
        e.tol_ritz = d.tol_ritz;
        e.tol_res = d.tol_res;
        e.max_ws = d.max_wave_solves;
        e.seed = d.seed;
        e.v0 = d.v0_dev;
        e.ws.stream = b->user_stream;
        e.ws.g = b->P[i].g;
        e.ws.order = b->order;
        EW_TRY(e.ws.setup(N, d.m, d.k));
    }
    // batched Gram-Schmidt tables
    std::vector<int> mgs_starts(np + 1, 0);
    std::vector<int> part_off(np), hmax(np), h_off(np);
    int part_total = 0, h_total = 0;
    for (int i = 0; i < np; ++i) {
        const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, (b->P[i].N + 4095) / 4096));
        mgs_starts[i + 1] = mgs_starts[i] + nb;
        part_off[i] = part_total;
        part_total += 2 * nb;
        hmax[i] = E[i]->ws.cap_lock + E[i]->m + 2;
        h_off[i] = h_total;
        h_total += hmax[i];
    }
    const int lmax_all = *std::max_element(hmax.begin(), hmax.end());
    double *partial = nullptr, *hout = nullptr;
    int* mgs_blk = nullptr;
    BatchMgsDev* info_dev = nullptr;
    MgsLink* links_dev = nullptr;
    std::vector<void*> tmp;
    auto talloc = [&](void** p, size_t bytes) -> ew_status {
        hipError_t e = dev_alloc(p, bytes, b->user_stream);
        if (e != hipSuccess) return fail(EW_ERR_OOM, "batch eigensolver tables");
        tmp.push_back(*p);
        return EW_OK;
    };
    struct Cleanup {
        std::vector<void*>& t;
        ~Cleanup() {
            for (void* p : t) dev_free(p);
        }
    } cleanup{tmp};
    EW_TRY(talloc((void**)&partial, part_total * sizeof(double)));
    EW_TRY(talloc((void**)&hout, h_total * sizeof(double)));
    EW_TRY(talloc((void**)&mgs_blk, (np + 1) * sizeof(int)));
    EW_TRY(talloc((void**)&info_dev, np * sizeof(BatchMgsDev)));
    EW_TRY(talloc((void**)&links_dev, (size_t)lmax_all * np * sizeof(MgsLink)));
    EW_HIP_TRY(hipMemcpy(mgs_blk, mgs_starts.data(), (np + 1) * sizeof(int), hipMemcpyHostToDevice));
    std::vector<BatchMgsDev> info(np);
    std::vector<MgsLink> links((size_t)lmax_all * np);
    std::vector<double> hhost(h_total);
    std::vector<const double*> vptr(np);
    std::vector<double*> optr(np);
    std::vector<char> active(np);
    const int64_t ws0 = b->wave_solves, pt0 = b->pt_updates;
    std::vector<double> coeff;

    for (;;) {
        // start new runs
        for (int i = 0; i < np; ++i) {
            BEig& e = *E[i];
            if (e.phase == 0 && e.status == EW_OK) {
                if (e.wave_solves >= e.max_ws) {
                    e.budget_hit = true;
                    e.phase = 2;
                    continue;
                }
                ew_status st = start_run(e);
                if (st != EW_OK) {
                    e.status = st;
                    e.phase = 2;
                }
            }
        }
        int nact = 0, lmax = 0;
        for (int i = 0; i < np; ++i) {
            BEig& e = *E[i];
            active[i] = 0;
            if (e.phase != 1) continue;
            if (e.wave_solves >= e.max_ws) {  // budget reached inside a cycle
                e.budget_hit = true;
                e.phase = 2;
                continue;
            }
            active[i] = 1;
            ++nact;
            lmax = std::max(lmax, e.nl + e.j + 1);
        }
        if (nact == 0) break;
        for (int i = 0; i < np; ++i) {
            BEig& e = *E[i];
            vptr[i] = e.phase == 1 ? e.ws.col(e.ws.V, e.j) : e.ws.V;
            optr[i] = e.phase == 1 ? e.ws.col(e.ws.V, e.j + 1) : e.ws.Vt;
        }
        EW_TRY(batch_apply(b, vptr.data(), optr.data(), active.data()));
        // batched Gram-Schmidt: chain over the locked vectors, then V[:, 0..j]
        for (int i = 0; i < np; ++i) {
            BEig& e = *E[i];
            BatchMgsDev& I = info[i];
            I.n = b->P[i].N;
            I.nblk = mgs_starts[i + 1] - mgs_starts[i];
            I.part_off = part_off[i];
            I.h_off = h_off[i];
            if (!active[i]) {
                I.q = -1;
                I.w = nullptr;
                continue;
            }
            const int nu = e.nl + e.j + 1;
            I.q = nu + 1;
            I.w = e.ws.col(e.ws.V, e.j + 1);
            for (int l = 0; l < nu; ++l)
                links[(size_t)l * np + i].u = l < e.nl ? e.ws.col(e.ws.Y, l) : e.ws.col(e.ws.V, l - e.nl);
        }
        EW_HIP_TRY(hipMemcpyAsync(info_dev, info.data(), np * sizeof(BatchMgsDev), hipMemcpyHostToDevice, b->user_stream));
        EW_HIP_TRY(hipMemcpyAsync(links_dev, links.data(), (size_t)lmax * np * sizeof(MgsLink), hipMemcpyHostToDevice,
                                  b->user_stream));
        for (int ell = 0; ell <= lmax + 1; ++ell)
            EW_HIP_TRY(launch_batch_mgs(info_dev, links_dev, np, mgs_blk, mgs_starts[np], ell, partial, hout,
                                        b->user_stream));
        EW_HIP_TRY(hipMemcpyAsync(hhost.data(), hout, h_total * sizeof(double), hipMemcpyDeviceToHost, b->user_stream));
        EW_HIP_TRY(hipStreamSynchronize(b->user_stream));
        // per-problem bookkeeping
        for (int i = 0; i < np; ++i) {
            if (!active[i]) continue;
            BEig& e = *E[i];
            e.wave_solves++;
            e.pt_updates += b->P[i].N * (int64_t)b->P[i].tp.n_t;
            const int nu = e.nl + e.j + 1;
            const double* hc = hhost.data() + h_off[i];
            double hsq = 0.0;
            for (int r = 0; r <= e.j; ++r) {
                e.T(r, e.j) = hc[e.nl + r];
                hsq += hc[e.nl + r] * hc[e.nl + r];
            }
            double nrm = hc[nu];
            if (!std::isfinite(nrm) || !std::isfinite(hsq)) {
                e.status = fail(EW_ERR_NONFINITE, "non-finite value in Gram-Schmidt");
                e.phase = 2;
                continue;
            }
            if (!(nrm > 1e-12 * std::sqrt(hsq + nrm * nrm))) {
                // breakdown: continue from a fresh direction orthogonal to everything so far
                double* w = e.ws.col(e.ws.V, e.j + 1);
                EW_HIP_TRY(launch_splitmix_uniform(w, e.ws.N, e.seed + 0x100000ULL + (uint64_t)e.wave_solves, e.ws.stream));
                std::vector<const double*> u;
                for (int l = 0; l < e.nl; ++l) u.push_back(e.ws.col(e.ws.Y, l));
                for (int l = 0; l <= e.j; ++l) u.push_back(e.ws.col(e.ws.V, l));
                EW_TRY(mgs_orthonormalize(e.ws, w, u, coeff));
                nrm = 0.0;
            }
            e.T(e.j + 1, e.j) = nrm;
            e.j++;
            if (e.j == e.m) {
                bool ended = false;
                std::vector<double> theta;
                Mat Q;
                std::vector<char> conv;
                EW_TRY(end_of_cycle(e, ended, theta, Q, conv));
                if (ended) EW_TRY(finish_run(e, theta, Q, conv));
            }
        }
    }
    // Stage 2 per problem
    ew_status overall = EW_OK;
    int64_t ws_total = 0, rs_total = 0, runs_total = 0;
    double max_res = 0.0;
    int n_conv_total = 0;
    for (int i = 0; i < np; ++i) {
        BEig& e = *E[i];
        ws_total += e.wave_solves;
        rs_total += e.restarts;
        runs_total += e.runs;
        int nc = 0, nr = 0;
        double mr = 0.0;
        if (e.status == EW_OK && e.nl >= e.k) {
            EW_TRY(stage2(e.ws, e.nl, e.th_locked, e.tol_res, k_cap, mu_host ? mu_host + (size_t)i * k_cap : nullptr,
                          beta_host ? beta_host + (size_t)i * k_cap : nullptr,
                          res_host ? res_host + (size_t)i * k_cap : nullptr, Y_dev ? Y_dev[i] : nullptr, &nc, &nr, &mr));
            if (e.budget_hit) overall = EW_ERR_NOT_CONVERGED;
        } else {
            overall = e.status != EW_OK ? e.status : EW_ERR_NOT_CONVERGED;
        }
        if (n_conv_host) n_conv_host[i] = nc;
        n_conv_total += nc;
        max_res = std::max(max_res, mr);
    }
    EW_HIP_TRY(hipStreamSynchronize(b->user_stream));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n_conv = n_conv_total;
        stats->n_returned = 0;
        stats->wave_solves = ws_total;
        stats->restarts = rs_total;
        stats->probes = runs_total;
        stats->time_steps = 0;
        for (int i = 0; i < np; ++i) stats->time_steps += E[i]->wave_solves * (int64_t)b->P[i].tp.n_t;
        stats->pt_updates = b->pt_updates - pt0;
        stats->mg_cycles = 0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->max_res = max_res;
    }
    (void)ws0;
    if (overall != EW_OK) return fail(overall, "batched eigensolver: some problems did not converge");
    return EW_OK;
}
