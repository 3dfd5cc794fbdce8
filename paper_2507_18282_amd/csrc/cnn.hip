// Learned warm start for the implicit solves: the network object (FP32
// master parameters, Adam state, the packed BF16 image), the crop store, data
// collection from wave-solves, training on the residual loss, and the
// correction of the base guess used by the implicit step.  All arithmetic
// runs in cnn_kernels.hip and the multigrid's residual kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "cnn.h"
#include "op.h"

namespace ew {

struct Cnn {
    int device = 0;
    hipStream_t stream = nullptr;
    float* params = nullptr;  // FP32 master
    float* m = nullptr;       // Adam first moment
    float* v = nullptr;       // Adam second moment
    float* grad = nullptr;
    CnnPacked* pk = nullptr;
    float* pgrad = nullptr;   // kCnnTrainBlocks x kCnnParams partials
    double* ploss = nullptr;  // kCnnTrainBlocks
    double* loss_dev = nullptr;
    double* loss_host = nullptr;
    int* ids_dev = nullptr;
    int ids_cap = 0;
    // per-batch outputs, residuals and dL/dy of the residual loss
    float* ybuf = nullptr;
    float* ebuf = nullptr;
    float* dybuf = nullptr;
    int64_t batch_cap = 0;     // elements of each of the three
    int64_t adam_t = 0;
    std::vector<void*> allocations;

    ~Cnn() {
        for (void* p : allocations) dev_free(p);
        if (loss_host) hipHostFree(loss_host);
    }
    ew_status alloc(void** p, size_t bytes) {
        hipError_t e = dev_alloc(p, bytes, stream);
        if (e != hipSuccess) {
            *p = nullptr;
            return fail(EW_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        allocations.push_back(*p);
        return EW_OK;
    }
    ew_status ensure_batch(int64_t elems) {
        if (elems <= batch_cap) return EW_OK;
        EW_TRY(alloc((void**)&ybuf, (size_t)elems * sizeof(float)));
        EW_TRY(alloc((void**)&ebuf, (size_t)elems * sizeof(float)));
        EW_TRY(alloc((void**)&dybuf, (size_t)elems * sizeof(float)));
        batch_cap = elems;
        return EW_OK;
    }
    ew_status ensure_ids(int n) {
        if (n <= ids_cap) return EW_OK;
        void* p = nullptr;
        EW_TRY(alloc(&p, (size_t)n * sizeof(int)));
        ids_dev = (int*)p;
        ids_cap = n;
        return EW_OK;
    }
};

struct CnnData {
    int device = 0;
    int capacity = 0, crop = 0, count = 0;
    int order = 4;             // stencil order of the steps' M
    float* fields = nullptr;   // [capacity][2][crop+6][crop+6]
    float* target = nullptr;   // [capacity][crop][crop]
    CropMeta* meta = nullptr;  // [capacity]
    int* origins_dev = nullptr;
    int origins_cap = 0;
    uint64_t draws = 0;        // SplitMix64 counter of the window origins
    std::vector<void*> allocations;

    ~CnnData() {
        for (void* p : allocations) dev_free(p);
    }
    int64_t field_elems() const { return 2LL * (crop + 2 * kCnnHalo) * (crop + 2 * kCnnHalo); }
    int64_t target_elems() const { return (int64_t)crop * crop; }
};

namespace {

// SplitMix64 (Steele, Lea and Flood 2014) in counter form: output i of stream
// `seed` mixes seed + (i + 1) * golden gamma; uniform in [0,1) from the top 53 bits.
uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
double unit_at(uint64_t seed, uint64_t i) { return (double)(splitmix64_at(seed, i) >> 11) * 0x1.0p-53; }

// Constant input planes of an implicit step with M = I - a L.
void step_planes(double a, double omega, double h, float* c2, float* c3) {
    const double aw2 = a * omega * omega;
    *c2 = (float)(aw2 / (1.0 + aw2));
    *c3 = (float)(std::fmin(a / (h * h), 100.0) / 100.0);
}

ew_status check_cnn_op(Op* op) {
    if (op->dim != 2) return fail(EW_ERR_UNSUPPORTED, "the learned guess is implemented for 2D grids");
    if (!op->implicit) return fail(EW_ERR_INVALID_ARG, "the learned guess needs an implicit operator");
    if (op->n[0] > (1 << 30) / op->n[1]) return fail(EW_ERR_INVALID_ARG, "grid too large for int indexing");
    return EW_OK;
}

ew_status upload_ids(Cnn* c, const std::vector<int>& ids) {
    EW_TRY(c->ensure_ids((int)ids.size()));
    EW_HIP_TRY(hipMemcpyAsync(c->ids_dev, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    return EW_OK;
}

ew_status check_range(CnnData* d, int first, int count) {
    if (first < 0 || count <= 0 || first > d->count - count)
        return fail(EW_ERR_INVALID_ARG, "crop range outside the filled part of the store");
    return EW_OK;
}

// One pass over ids[0..count) of d: mode 0 writes the network outputs to
// y_out; mode 1 forms the outputs, the residual loss and dL/dy
// (k_cnn_resid, k_cnn_resgrad), backpropagates, and reduces the gradient and
// the loss (mean over the batch's window points of e^2).
ew_status train_pass(Cnn* c, CnnData* d, const int* ids_dev, int count, int mode, float* y_out, float* grad,
                     double* loss_dev) {
    const int nb = cnn_train_blocks(count, d->crop);
    const float inv_npix = (float)(1.0 / ((double)count * d->crop * d->crop));
    if (mode == 0) {
        EW_HIP_TRY(launch_cnn_train(c->pk, d->fields, d->meta, ids_dev, count, d->crop, 0, y_out, nullptr, nullptr,
                                    inv_npix, c->pgrad, c->ploss, nb, c->stream));
        return EW_OK;
    }
    EW_TRY(c->ensure_batch((int64_t)count * d->crop * d->crop));
    EW_HIP_TRY(launch_cnn_train(c->pk, d->fields, d->meta, ids_dev, count, d->crop, 0, c->ybuf, nullptr, nullptr,
                                inv_npix, c->pgrad, c->ploss, nb, c->stream));
    EW_HIP_TRY(launch_cnn_resloss(c->ybuf, d->target, d->meta, ids_dev, count, d->crop, inv_npix, c->ebuf, c->dybuf,
                                  c->stream));
    EW_HIP_TRY(launch_cnn_train(c->pk, d->fields, d->meta, ids_dev, count, d->crop, 1, nullptr, c->dybuf, c->ebuf,
                                inv_npix, c->pgrad, c->ploss, nb, c->stream));
    EW_HIP_TRY(launch_cnn_reduce(c->pgrad, c->ploss, nb, grad, loss_dev, c->stream));
    return EW_OK;
}

// ||bscale b||^2 from the value the projection guess left for b, or a reduction.
ew_status rhs_sq(Op* op, const double* b, double bscale, double* out) {
    double bb;
    if (op->bb_src == b) {
        bb = op->bb_val;
    } else {
        EW_HIP_TRY(launch_dot_partial(b, b, op->N, op->partial_dev, op->stream));
        EW_TRY(op->host_sum_partials(&bb));
        op->bb_src = b;
        op->bb_val = bb;
    }
    if (!std::isfinite(bb)) return fail(EW_ERR_NONFINITE, "non-finite right-hand side");
    *out = bb * bscale * bscale;
    return EW_OK;
}

}  // namespace

// The network's correction of the base guess x of M x = bscale b:
// r = bscale b - M x, then x += s y with y = network(r / s, b / s_b, c2, c3),
// s = RMS(r) (read on the device from the residual's norm partials), s_b =
// RMS(bscale b).  x must hold the base guess (zero filled by the caller).
ew_status cnn_correct(Op* op, const double* b, double bscale, double* x) {
    Cnn* c = op->cnn;
    if (!c) return fail(EW_ERR_INVALID_ARG, "no network attached");
    double bb = 0.0;
    EW_TRY(rhs_sq(op, b, bscale, &bb));
    if (bb == 0.0) return EW_OK;
    const double sb = std::sqrt(bb / (double)op->N);
    EW_HIP_TRY((launch_residual_tile<double, double>(x, b, bscale, op->g, op->order, op->a, op->tile_partial_dev,
                                                     op->partial_dev, op->cnn_r, op->stream)));
    float c2, c3;
    step_planes(op->a, op->omega_used, op->h[0], &c2, &c3);
    EW_HIP_TRY(launch_cnn_infer(c->pk, op->cnn_r, b, x, (int)op->n[0], (int)op->n[1], op->partial_dev,
                                1.0 / (double)op->N, bscale / sb, c2, c3, op->stream));
    op->stats.cnn_guesses++;
    return EW_OK;
}

}  // namespace ew

using namespace ew;

struct ew_cnn_s : public Cnn {};
struct ew_cnn_data_s : public CnnData {};

extern "C" ew_status ew_cnn_create(uint64_t seed, void* hip_stream, ew_cnn* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    std::unique_ptr<ew_cnn_s> c(new ew_cnn_s());
    c->stream = (hipStream_t)hip_stream;
    EW_HIP_TRY(hipGetDevice(&c->device));
    EW_TRY(c->alloc((void**)&c->params, kCnnParams * sizeof(float)));
    EW_TRY(c->alloc((void**)&c->m, kCnnParams * sizeof(float)));
    EW_TRY(c->alloc((void**)&c->v, kCnnParams * sizeof(float)));
    EW_TRY(c->alloc((void**)&c->grad, kCnnParams * sizeof(float)));
    EW_TRY(c->alloc((void**)&c->pk, sizeof(CnnPacked)));
    EW_TRY(c->alloc((void**)&c->pgrad, (size_t)kCnnTrainBlocks * kCnnParams * sizeof(float)));
    EW_TRY(c->alloc((void**)&c->ploss, kCnnTrainBlocks * sizeof(double)));
    EW_HIP_TRY(hipHostMalloc((void**)&c->loss_host, 2 * sizeof(double), hipHostMallocDefault));
    // He-uniform initialisation of the two hidden layers, W = u sqrt(6 / fan_in);
    // the last layer and the biases start at zero, so that the untrained
    // network returns the base guess (a He-scaled last layer starts from
    // residuals hundreds of times the base's, from which training on the
    // residual loss settles on a zero output instead of a correction).
    std::vector<float> init(kCnnParams, 0.f);
    struct Block { int off, n, fan_in; };
    const Block blocks[2] = {{kOffW1, 576, 4 * 9}, {kOffW2, 2304, 16 * 9}};
    for (const Block& b : blocks)
        for (int i = b.off; i < b.off + b.n; ++i)
            init[i] = (float)((2.0 * unit_at(seed, (uint64_t)i) - 1.0) * std::sqrt(6.0 / b.fan_in));
    ew_cnn raw = c.release();
    ew_status st = ew_cnn_set_params(raw, init.data());
    if (st != EW_OK) {
        delete raw;
        return st;
    }
    *out = raw;
    return EW_OK;
}

extern "C" void ew_cnn_destroy(ew_cnn cnn) { delete cnn; }

extern "C" ew_status ew_cnn_set_params(ew_cnn c, const float* params_host) {
    if (!c || !params_host) return fail(EW_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < kCnnParams; ++i)
        if (!std::isfinite(params_host[i])) return fail(EW_ERR_NONFINITE, "non-finite parameter");
    EW_HIP_TRY(hipMemcpyAsync(c->params, params_host, kCnnParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    EW_HIP_TRY(hipMemsetAsync(c->m, 0, kCnnParams * sizeof(float), c->stream));
    EW_HIP_TRY(hipMemsetAsync(c->v, 0, kCnnParams * sizeof(float), c->stream));
    EW_HIP_TRY(launch_cnn_pack(c->params, c->pk, c->stream));
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    return EW_OK;
}

extern "C" ew_status ew_cnn_get_params(ew_cnn c, float* params_host) {
    if (!c || !params_host) return fail(EW_ERR_INVALID_ARG, "null argument");
    EW_HIP_TRY(hipMemcpyAsync(params_host, c->params, kCnnParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    return EW_OK;
}

extern "C" ew_status ew_cnn_data_create(int capacity, int crop, int order, ew_cnn_data* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (capacity <= 0) return fail(EW_ERR_INVALID_ARG, "capacity must be positive");
    if (crop < 16 || crop > 256 || crop % 16 != 0) return fail(EW_ERR_INVALID_ARG, "crop must be a multiple of 16 in [16, 256]");
    if (order != 2 && order != 4) return fail(EW_ERR_INVALID_ARG, "order must be 2 or 4");
    std::unique_ptr<ew_cnn_data_s> d(new ew_cnn_data_s());
    EW_HIP_TRY(hipGetDevice(&d->device));
    d->capacity = capacity;
    d->crop = crop;
    d->order = order;
    const size_t fb = (size_t)capacity * d->field_elems() * sizeof(float);
    const size_t tb = (size_t)capacity * d->target_elems() * sizeof(float);
    void* p = nullptr;
    for (auto req : {std::make_pair((void**)&d->fields, fb), std::make_pair((void**)&d->target, tb),
                     std::make_pair((void**)&d->meta, (size_t)capacity * sizeof(CropMeta))}) {
        hipError_t e = dev_alloc(&p, req.second, nullptr);
        if (e != hipSuccess) return fail(EW_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        d->allocations.push_back(p);
        *req.first = p;
    }
    *out = d.release();
    return EW_OK;
}

extern "C" void ew_cnn_data_destroy(ew_cnn_data d) { delete d; }

extern "C" ew_status ew_cnn_data_count(ew_cnn_data d, int* count) {
    if (!d || !count) return fail(EW_ERR_INVALID_ARG, "null argument");
    *count = d->count;
    return EW_OK;
}

extern "C" ew_status ew_cnn_data_append(ew_cnn_data d, int n, const float* fields_dev, const float* target_dev,
                                        const float* planes_host, const int* rect_host) {
    if (!d || !fields_dev || !target_dev || !planes_host || !rect_host) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (n <= 0 || n > d->capacity - d->count) return fail(EW_ERR_INVALID_ARG, "n exceeds the free capacity");
    const int CP = d->crop + 2 * kCnnHalo;
    std::vector<CropMeta> meta(n);
    for (int i = 0; i < n; ++i) {
        CropMeta& m = meta[i];
        m.c2 = planes_host[4 * i];
        m.c3 = planes_host[4 * i + 1];
        m.ahx = planes_host[4 * i + 2];
        m.ahy = planes_host[4 * i + 3];
        m.order = d->order;
        m.pad = 0;
        if (!(m.ahx >= 0.f) || !(m.ahy >= 0.f) || !std::isfinite(m.ahx) || !std::isfinite(m.ahy))
            return fail(EW_ERR_INVALID_ARG, "a / h^2 must be finite and >= 0");
        m.r0 = rect_host[4 * i];
        m.r1 = rect_host[4 * i + 1];
        m.c0 = rect_host[4 * i + 2];
        m.c1 = rect_host[4 * i + 3];
        if (m.r0 < 0 || m.r1 > CP || m.r0 > m.r1 || m.c0 < 0 || m.c1 > CP || m.c0 > m.c1)
            return fail(EW_ERR_INVALID_ARG, "crop rectangle outside the padded window");
    }
    EW_HIP_TRY(hipMemcpy(d->fields + (int64_t)d->count * d->field_elems(), fields_dev,
                         (size_t)n * d->field_elems() * sizeof(float), hipMemcpyDeviceToDevice));
    EW_HIP_TRY(hipMemcpy(d->target + (int64_t)d->count * d->target_elems(), target_dev,
                         (size_t)n * d->target_elems() * sizeof(float), hipMemcpyDeviceToDevice));
    EW_HIP_TRY(hipMemcpy(d->meta + d->count, meta.data(), n * sizeof(CropMeta), hipMemcpyHostToDevice));
    d->count += n;
    return EW_OK;
}

extern "C" ew_status ew_cnn_data_read(ew_cnn_data d, int first, int count, float* fields_dev, float* target_dev,
                                      float* planes_host, int* rect_host) {
    if (!d) return fail(EW_ERR_INVALID_ARG, "null store");
    EW_TRY(check_range(d, first, count));
    if (fields_dev)
        EW_HIP_TRY(hipMemcpy(fields_dev, d->fields + (int64_t)first * d->field_elems(),
                             (size_t)count * d->field_elems() * sizeof(float), hipMemcpyDeviceToDevice));
    if (target_dev)
        EW_HIP_TRY(hipMemcpy(target_dev, d->target + (int64_t)first * d->target_elems(),
                             (size_t)count * d->target_elems() * sizeof(float), hipMemcpyDeviceToDevice));
    if (planes_host || rect_host) {
        std::vector<CropMeta> meta(count);
        EW_HIP_TRY(hipMemcpy(meta.data(), d->meta + first, count * sizeof(CropMeta), hipMemcpyDeviceToHost));
        for (int i = 0; i < count; ++i) {
            if (planes_host) {
                planes_host[4 * i] = meta[i].c2;
                planes_host[4 * i + 1] = meta[i].c3;
                planes_host[4 * i + 2] = meta[i].ahx;
                planes_host[4 * i + 3] = meta[i].ahy;
            }
            if (rect_host) {
                rect_host[4 * i] = meta[i].r0;
                rect_host[4 * i + 1] = meta[i].r1;
                rect_host[4 * i + 2] = meta[i].c0;
                rect_host[4 * i + 3] = meta[i].c1;
            }
        }
    }
    return EW_OK;
}

extern "C" ew_status ew_cnn_data_collect(ew_cnn_data d, ew_op op, const double* v_dev, double* out_dev,
                                         int crops_per_step, uint64_t seed) {
    if (!d || !op || !v_dev || !out_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (v_dev == out_dev) return fail(EW_ERR_INVALID_ARG, "v and out may not alias");
    EW_TRY(check_cnn_op(op));
    if (op->mixed) return fail(EW_ERR_UNSUPPORTED, "crops are collected from FP64 operators");
    if (op->order != d->order) return fail(EW_ERR_INVALID_ARG, "the operator's order differs from the store's");
    if (crops_per_step <= 0) return fail(EW_ERR_INVALID_ARG, "crops_per_step must be positive");
    const int nx = (int)op->n[0], ny = (int)op->n[1], crop = d->crop;
    if (nx < crop || ny < crop) return fail(EW_ERR_INVALID_ARG, "grid smaller than the crop");
    if (d->origins_cap < crops_per_step) {
        void* p = nullptr;
        hipError_t e = dev_alloc(&p, (size_t)crops_per_step * 2 * sizeof(int), op->stream);
        if (e != hipSuccess) return fail(EW_ERR_OOM, "hipMalloc of crop origins failed");
        d->allocations.push_back(p);
        d->origins_dev = (int*)p;
        d->origins_cap = crops_per_step;
    }
    // the base guess's residual of each step, for this call only
    double* rbuf = nullptr;
    {
        void* p = nullptr;
        hipError_t e = dev_alloc(&p, (size_t)op->N * sizeof(double), op->stream);
        if (e != hipSuccess) return fail(EW_ERR_OOM, "hipMalloc of the residual buffer failed");
        rbuf = (double*)p;
    }
    struct FreeOnExit {
        void* p;
        hipStream_t s;
        ~FreeOnExit() {
            (void)hipStreamSynchronize(s);
            dev_free(p);
        }
    } free_rbuf{rbuf, op->stream};
    float c2, c3;
    step_planes(op->a, op->omega_used, op->h[0], &c2, &c3);
    const float ahx = (float)(op->a / (op->h[0] * op->h[0])), ahy = (float)(op->a / (op->h[1] * op->h[1]));
    const int CP = crop + 2 * kCnnHalo;
    // origin along an axis of n points: one eighth of the range beyond each end clamps to the wall
    auto origin = [&](int n) {
        const int range = n - crop + 1;
        const int extra = range / 8;
        const double u = unit_at(seed, d->draws++);
        int o = (int)std::floor(u * (double)(range + 2 * extra)) - extra;
        return o < 0 ? 0 : (o > range - 1 ? range - 1 : o);
    };
    // At every solve M x = bscale b of a step n >= 1, once the operator's base
    // guess x0 is formed (before the multigrid): r = bscale b - M x0, crops of
    // (r / s, bscale b / s_b) and the target r / s.
    op->guess_hook = [&](const double* b, double bscale, double* x0, bool x_is_zero) -> ew_status {
        if (x_is_zero) EW_HIP_TRY(launch_fill<double>(x0, op->N, 0.0, op->stream));
        const int k = std::min(crops_per_step, d->capacity - d->count);
        if (k <= 0) return EW_OK;
        double bb = 0.0;
        EW_TRY(rhs_sq(op, b, bscale, &bb));
        if (!(bb > 0.0)) return EW_OK;  // nothing to learn from a zero right-hand side
        EW_HIP_TRY((launch_residual_tile<double, double>(x0, b, bscale, op->g, op->order, op->a, op->tile_partial_dev,
                                                         op->partial_dev, rbuf, op->stream)));
        double rr = 0.0;
        EW_TRY(op->host_sum_partials(&rr));
        if (!(rr > 0.0) || !std::isfinite(rr)) return EW_OK;  // an exact base guess: nothing to correct
        const double s = std::sqrt(rr / (double)op->N), sb = std::sqrt(bb / (double)op->N);
        std::vector<int> org(2 * k);
        std::vector<CropMeta> meta(k);
        for (int j = 0; j < k; ++j) {
            const int oy = origin(ny), ox = origin(nx);
            org[2 * j] = oy;
            org[2 * j + 1] = ox;
            CropMeta& m = meta[j];
            m.c2 = c2;
            m.c3 = c3;
            m.r0 = std::max(0, kCnnHalo - oy);
            m.r1 = std::min(CP, ny - (oy - kCnnHalo));
            m.c0 = std::max(0, kCnnHalo - ox);
            m.c1 = std::min(CP, nx - (ox - kCnnHalo));
            m.ahx = ahx;
            m.ahy = ahy;
            m.order = d->order;
            m.pad = 0;
        }
        EW_HIP_TRY(hipMemcpyAsync(d->origins_dev, org.data(), org.size() * sizeof(int), hipMemcpyHostToDevice,
                                  op->stream));
        EW_HIP_TRY(hipMemcpyAsync(d->meta + d->count, meta.data(), k * sizeof(CropMeta), hipMemcpyHostToDevice,
                                  op->stream));
        EW_HIP_TRY(launch_cnn_extract(rbuf, b, nx, ny, 1.0 / s, bscale / sb, d->origins_dev, k, crop,
                                      d->fields + (int64_t)d->count * d->field_elems(),
                                      d->target + (int64_t)d->count * d->target_elems(), op->stream));
        // the host vectors above are read by the copies: finish before they go out of scope
        EW_HIP_TRY(hipStreamSynchronize(op->stream));
        d->count += k;
        return EW_OK;
    };
    ew_status st = op->apply_filter(v_dev, out_dev);
    op->guess_hook = nullptr;
    if (st != EW_OK) return st;
    EW_HIP_TRY(hipStreamSynchronize(op->stream));
    return EW_OK;
}

extern "C" ew_status ew_cnn_forward(ew_cnn c, ew_cnn_data d, int first, int count, float* y_dev) {
    if (!c || !d || !y_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    EW_TRY(check_range(d, first, count));
    std::vector<int> ids(count);
    for (int i = 0; i < count; ++i) ids[i] = first + i;
    EW_TRY(upload_ids(c, ids));
    EW_TRY(train_pass(c, d, c->ids_dev, count, 0, y_dev, nullptr, nullptr));
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    return EW_OK;
}

extern "C" ew_status ew_cnn_loss_grad(ew_cnn c, ew_cnn_data d, int first, int count, double* loss_host,
                                      float* grad_dev) {
    if (!c || !d || !grad_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    EW_TRY(check_range(d, first, count));
    std::vector<int> ids(count);
    for (int i = 0; i < count; ++i) ids[i] = first + i;
    EW_TRY(upload_ids(c, ids));
    if (!c->loss_dev) EW_TRY(c->alloc((void**)&c->loss_dev, sizeof(double)));
    EW_TRY(train_pass(c, d, c->ids_dev, count, 1, nullptr, grad_dev, c->loss_dev));
    EW_HIP_TRY(hipMemcpyAsync(c->loss_host, c->loss_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    if (loss_host) *loss_host = c->loss_host[0];
    return EW_OK;
}

extern "C" ew_status ew_cnn_train(ew_cnn c, ew_cnn_data d, const ew_cnn_train_desc* desc, ew_cnn_train_stats* stats) {
    if (!c || !d || !desc) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (desc->steps <= 0 || desc->batch <= 0) return fail(EW_ERR_INVALID_ARG, "steps and batch must be positive");
    if (d->count <= 0) return fail(EW_ERR_INVALID_ARG, "the crop store is empty");
    if (!(desc->lr > 0) || !(desc->beta1 >= 0 && desc->beta1 < 1) || !(desc->beta2 >= 0 && desc->beta2 < 1) ||
        !(desc->eps > 0))
        return fail(EW_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    const int64_t nids = (int64_t)desc->steps * desc->batch;
    if (nids > (1 << 26)) return fail(EW_ERR_INVALID_ARG, "steps x batch too large");
    std::vector<int> ids((size_t)nids);
    for (int64_t i = 0; i < nids; ++i) {
        int k = (int)std::floor(unit_at(desc->seed, (uint64_t)i) * d->count);
        ids[i] = k < d->count ? k : d->count - 1;
    }
    EW_TRY(upload_ids(c, ids));
    void* lp = nullptr;
    EW_TRY(c->alloc(&lp, (size_t)desc->steps * sizeof(double)));
    double* losses = (double*)lp;
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    for (int s = 0; s < desc->steps; ++s) {
        EW_TRY(train_pass(c, d, c->ids_dev + (int64_t)s * desc->batch, desc->batch, 1, nullptr, c->grad, losses + s));
        const int64_t t = ++c->adam_t;
        const double ic1 = 1.0 / (1.0 - std::pow(desc->beta1, (double)t));
        const double ic2 = 1.0 / (1.0 - std::pow(desc->beta2, (double)t));
        EW_HIP_TRY(launch_cnn_adam_pack(c->params, c->m, c->v, c->grad, (float)desc->lr, (float)desc->beta1,
                                        (float)desc->beta2, (float)desc->eps, (float)ic1, (float)ic2, c->pk,
                                        c->stream));
    }
    EW_HIP_TRY(hipMemcpyAsync(c->loss_host, losses, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    EW_HIP_TRY(hipMemcpyAsync(c->loss_host + 1, losses + desc->steps - 1, sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    EW_HIP_TRY(hipStreamSynchronize(c->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // release the per-call loss log (the batch buffers the steps may have
    // added after it stay with the network)
    c->allocations.erase(std::find(c->allocations.begin(), c->allocations.end(), lp));
    dev_free(lp);
    if (stats) {
        stats->steps = desc->steps;
        stats->first_loss = c->loss_host[0];
        stats->last_loss = c->loss_host[1];
        stats->seconds = secs;
    }
    return EW_OK;
}

extern "C" ew_status ew_op_set_cnn(ew_op op, ew_cnn cnn) {
    if (!op) return fail(EW_ERR_INVALID_ARG, "null operator");
    if (cnn) {
        EW_TRY(check_cnn_op(op));
        if (op->mixed) return fail(EW_ERR_UNSUPPORTED, "the learned guess corrects FP64 solves");
        if (!op->cnn_r) EW_TRY(op->alloc((void**)&op->cnn_r, (size_t)op->N * sizeof(double)));
    }
    op->cnn = cnn;
    return EW_OK;
}

extern "C" ew_status ew_op_cnn_guess(ew_op op, const double* b_dev, double* base_dev, double* guess_dev) {
    if (!op || !b_dev || !guess_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    EW_TRY(check_cnn_op(op));
    if (!op->cnn) return fail(EW_ERR_INVALID_ARG, "no network attached");
    if (guess_dev == b_dev || base_dev == b_dev || (base_dev && base_dev == guess_dev))
        return fail(EW_ERR_INVALID_ARG, "b, base and guess may not alias");
    op->solve_kind = 1;
    bool zero = true;
    if (op->desc.predictor == EW_PRED_PROJ || op->desc.predictor == EW_PRED_CNN)
        EW_TRY(op->proj_guess(b_dev, 1.0, guess_dev, &zero));
    if (zero) EW_HIP_TRY(launch_fill<double>(guess_dev, op->N, 0.0, op->stream));
    if (base_dev)
        EW_HIP_TRY(hipMemcpyAsync(base_dev, guess_dev, op->N * sizeof(double), hipMemcpyDeviceToDevice, op->stream));
    EW_TRY(cnn_correct(op, b_dev, 1.0, guess_dev));
    // no solve follows: the projection keeps no pair for this right-hand side
    op->proj_rhs_ok = false;
    op->bb_src = nullptr;
    EW_HIP_TRY(hipStreamSynchronize(op->stream));
    return EW_OK;
}
