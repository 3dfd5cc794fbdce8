// ew_apply_filter_noalloc: the explicit wave-solve with time filter (S v of
// ew_op_apply_filter) for callers that cannot allocate device memory.  No
// operator object is created: the time plan is computed on the host from the
// descriptors and the time levels live in a file-scope device array that the
// library reserves once per GPU.
#include <mutex>

#include "op.h"

namespace ew {

// Scratch of the no-allocation wave-solve: 2^23 doubles (64 MiB) per GPU,
// held until the process ends.  FP64 runs use two time levels (2 N doubles),
// mixed runs four FP32 arrays (2 N doubles as well), so N <= 2^22 points.
constexpr size_t kNoAllocScratchDoubles = (size_t)1 << 23;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

// Device address of `scratch` on each GPU.  The array's name is a host-side
// stand-in in host code; every launch takes the address resolved here.
constexpr int kNoAllocMaxDevices = 64;
static double* g_scratch_dev[kNoAllocMaxDevices] = {};
static std::mutex g_scratch_mu;

static ew_status scratch_on_current_device(double** out) {
    int dev = 0;
    EW_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(EW_ERR_UNSUPPORTED, "ew_apply_filter_noalloc supports device ordinals below 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(EW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return EW_OK;
}

}  // namespace ew

using namespace ew;

extern "C" ew_status ew_apply_filter_noalloc(const ew_grid_desc* grid, const ew_op_desc* desc, const double* v_dev,
                                             double* out_dev, void* hip_stream) {
    if (!grid || !desc || !v_dev || !out_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (v_dev == out_dev) return fail(EW_ERR_INVALID_ARG, "v and out may not alias");
    EW_TRY(validate_descs(grid, desc));
    if (desc->ts != EW_TS_EXPLICIT)
        return fail(EW_ERR_UNSUPPORTED, "ew_apply_filter_noalloc runs explicit time stepping only");
    int64_t n[3];
    double len[3], h[3];
    int wall = 0;
    grid_geometry(grid, n, len, h, &wall);
    const Geo g = make_geo(grid->dim, n, h, wall);
    const int64_t N = g.size();
    if ((size_t)N > kNoAllocScratchDoubles / 2)
        return fail(EW_ERR_INVALID_ARG, "ew_apply_filter_noalloc: " + std::to_string(N) +
                                            " active points exceed its scratch limit of " +
                                            std::to_string(kNoAllocScratchDoubles / 2));
    double* scr = nullptr;
    EW_TRY(scratch_on_current_device(&scr));
    TimePlan tp;
    make_time_plan(grid->dim, grid->order, h, *desc, tp, 0.0, false);
    const hipStream_t s = (hipStream_t)hip_stream;
    const double dt2 = tp.dt * tp.dt;
    const int order = grid->order;
    // Every array below is written before it is read (the first step writes
    // W^1 and the accumulator whole), so nothing left by an earlier call
    // enters the result.
    if (desc->precision == EW_PREC_FP64) {
        double* wA = scr;
        double* wB = scr + N;
        EW_HIP_TRY(launch_leapfrog<double>(v_dev, nullptr, wA, out_dev, g, order, dt2, filter_weight(tp, 0),
                                           filter_weight(tp, 1), 1, s));
        const double* prev = v_dev;
        double* cur = wA;
        for (int k = 1; k < tp.n_t; ++k) {
            double* next = (prev == v_dev) ? wB : const_cast<double*>(prev);
            EW_HIP_TRY(launch_leapfrog<double>(cur, prev, next, out_dev, g, order, dt2, 0.0, filter_weight(tp, k + 1),
                                               0, s));
            prev = cur;
            cur = next;
        }
    } else {
        float* f0 = reinterpret_cast<float*>(scr);
        float* fA = f0 + N;
        float* fB = fA + N;
        float* acc = fB + N;
        EW_HIP_TRY((launch_convert<float, double>(f0, v_dev, N, 1.0, s)));
        EW_HIP_TRY(launch_leapfrog<float>(f0, nullptr, fA, acc, g, order, dt2, filter_weight(tp, 0),
                                          filter_weight(tp, 1), 1, s));
        float* prev = f0;
        float* cur = fA;
        for (int k = 1; k < tp.n_t; ++k) {
            float* next = (prev == f0) ? fB : prev;
            EW_HIP_TRY(launch_leapfrog<float>(cur, prev, next, acc, g, order, dt2, 0.0, filter_weight(tp, k + 1), 0, s));
            prev = cur;
            cur = next;
        }
        EW_HIP_TRY((launch_convert<double, float>(out_dev, acc, N, 1.0, s)));
    }
    return EW_OK;
}
