// ew_op: the WaveHoltz operator S (one wave-solve + trapezoidal time filter)
// on the device, with the implicit step's multigrid solver.
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "op.h"

namespace ew {

thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// Device allocator (ew_set_allocator): process-wide hooks and a count of the
// live blocks they handed out.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_alloc_mu;
ew_alloc_fn g_alloc = nullptr;
ew_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
std::atomic<int64_t> g_live_blocks{0};
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    *p = nullptr;
    ew_alloc_fn fa;
    void* ctx;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        fa = g_alloc;
        ctx = g_alloc_ctx;
    }
    if (fa) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        *p = fa(bytes, dev, (void*)s, ctx);
        if (!*p) return hipErrorOutOfMemory;
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            return e;
        }
    }
    g_live_blocks.fetch_add(1);
    return hipSuccess;
}

void dev_free(void* p) {
    if (!p) return;
    ew_free_fn ff;
    void* ctx;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        ff = g_free;
        ctx = g_alloc_ctx;
    }
    if (ff) {
        // hipFree waits for the device; a caller's allocator may hand the block
        // out again at once, so wait here for every kernel that may still use it.
        (void)hipDeviceSynchronize();
        ff(p, ctx);
    } else {
        hipFree(p);
    }
    g_live_blocks.fetch_sub(1);
}

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }
ew_status fail(ew_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

Geo make_geo(int dim, const int64_t* n, const double* h, int wall) {
    Geo g;
    g.dim = dim;
    g.wall = wall;
    g.nx = (int)n[0];
    g.ny = (int)n[1];
    g.nz = dim == 3 ? (int)n[2] : 1;
    g.ihx2 = 1.0 / (h[0] * h[0]);
    g.ihy2 = 1.0 / (h[1] * h[1]);
    g.ihz2 = dim == 3 ? 1.0 / (h[2] * h[2]) : 0.0;
    return g;
}

// ---------------------------------------------------------------------------
// Time plan (host, FP64), computed in the same order of operations as the
// definition: T_f = N_p 2 pi / omega; implicit N_t = N_p N_its; explicit
// dt_max = 2 / sqrt(rho), rho = sum_d c / h_d^2, N_t = ceil(T_f / (cfl dt_max));
// dt = T_f / N_t; c_n = (2/T_f) sigma_n (cos(omega n dt) - shift) with
// trapezoid weights sigma_0 = sigma_{N_t} = dt/2, dt otherwise, and
// shift = alpha_d/2 = tan(omega dt/2) / tan(omega dt) / 2 or 1/4.
// ---------------------------------------------------------------------------
void make_time_plan(int dim, int order, const double* h, const ew_op_desc& d, TimePlan& tp, double rho_override,
                    bool with_weights) {
    double om = d.omega;
    if (d.adjust_omega) {
        const double s = std::sin(M_PI / d.n_its);
        const double s2 = s * s;
        om = d.omega * M_PI / d.n_its * std::sqrt((1.0 - 2.0 * s2) / s2);
    }
    tp.omega_used = om;
    tp.t_final = d.n_p * 2.0 * M_PI / om;
    if (d.ts == EW_TS_IMPLICIT) {
        tp.n_t = d.n_p * d.n_its;
    } else {
        const double c = order == 2 ? 4.0 : 16.0 / 3.0;
        double rho = 0.0;
        for (int k = 0; k < dim; ++k) rho += c / (h[k] * h[k]);
        if (rho_override > 0.0) rho = rho_override;
        const double dt_max = 2.0 / std::sqrt(rho);
        tp.n_t = (int)std::ceil(tp.t_final / (d.cfl * dt_max));
    }
    tp.dt = tp.t_final / tp.n_t;
    tp.alpha_d = std::tan(om * tp.dt / 2.0) / std::tan(om * tp.dt);
    tp.shift = d.filter_const == EW_FILTER_ALPHA_D ? tp.alpha_d / 2.0 : 0.25;
    if (!with_weights) return;
    tp.c.resize(tp.n_t + 1);
    for (int k = 0; k <= tp.n_t; ++k) tp.c[k] = filter_weight(tp, k);
}

// c_k = (2 / T_f) sigma_k (cos(omega t_k) - shift), trapezoidal sigma_k.
double filter_weight(const TimePlan& tp, int k) {
    const double sigma = (k == 0 || k == tp.n_t) ? tp.dt / 2.0 : tp.dt;
    return (2.0 / tp.t_final) * sigma * (std::cos(tp.omega_used * k * tp.dt) - tp.shift);
}

static void make_plan(Op* op) {
    TimePlan tp;
    make_time_plan(op->dim, op->order, op->h, op->desc, tp);
    op->omega_used = tp.omega_used;
    op->t_final = tp.t_final;
    op->n_t = tp.n_t;
    op->dt = tp.dt;
    op->alpha_d = tp.alpha_d;
    op->c = tp.c;
}

Op::~Op() {
    for (void* p : allocations) dev_free(p);
    if (partial_host) hipHostFree(partial_host);
    if (proj_res_host) hipHostFree(proj_res_host);
    for (hipEvent_t e : prof.pool) hipEventDestroy(e);
}

ProfScope::ProfScope(Op* o, int kclass, int level, double bytes, bool external_events)
    : op(o), on(false), external(external_events) {
    Profiler& p = op->prof;
    if (!p.wants(kclass, level)) return;
    while (p.pool.size() < p.used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        p.pool.push_back(e);
    }
    if (!external && hipEventRecord(p.pool[p.used], op->stream) != hipSuccess) return;
    on = true;
    p.launches++;
    p.bytes += bytes;
}

hipEvent_t ProfScope::start_event() const { return on ? op->prof.pool[op->prof.used] : nullptr; }
hipEvent_t ProfScope::stop_event() const { return on ? op->prof.pool[op->prof.used + 1] : nullptr; }

ProfScope::~ProfScope() {
    if (!on) return;
    Profiler& p = op->prof;
    if (!external) hipEventRecord(p.pool[p.used + 1], op->stream);
    p.used += 2;
}

ew_status Op::alloc(void** p, size_t bytes) {
    hipError_t e = dev_alloc(p, bytes, stream);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(EW_ERR_OOM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed: " +
                                    hipGetErrorString(e));
    }
    allocations.push_back(*p);
    return EW_OK;
}

// Sum of the kRedBlocks partials on the host, in a fixed order.
ew_status Op::host_sum_partials(double* out) {
    EW_HIP_TRY(hipMemcpyAsync(partial_host, partial_dev, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, stream));
    EW_HIP_TRY(hipStreamSynchronize(stream));
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += partial_host[b];
    *out = s;
    return EW_OK;
}

ew_status validate_descs(const ew_grid_desc* g, const ew_op_desc* d) {
    if (!g || !d) return fail(EW_ERR_INVALID_ARG, "null descriptor");
    if (g->dim != 2 && g->dim != 3) return fail(EW_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (g->order != 2 && g->order != 4) return fail(EW_ERR_INVALID_ARG, "order must be 2 or 4");
    int64_t total = 1;
    bool neumann = false;
    for (int k = 0; k < g->dim; ++k) {
        if (g->n[k] < 1 || g->n[k] > 65535) return fail(EW_ERR_INVALID_ARG, "n[d] must be in [1, 65535]");
        if (!(g->len[k] > 0.0) || !std::isfinite(g->len[k])) return fail(EW_ERR_INVALID_ARG, "len[d] must be > 0");
        for (int e = 0; e < 2; ++e) {
            if (g->walls[k][e] != EW_WALL_DIRICHLET && g->walls[k][e] != EW_WALL_NEUMANN)
                return fail(EW_ERR_INVALID_ARG, "walls[d][e] must be EW_WALL_DIRICHLET or EW_WALL_NEUMANN");
            if (g->walls[k][e] == EW_WALL_NEUMANN) {
                neumann = true;
                if (g->n[k] < 3) return fail(EW_ERR_INVALID_ARG, "an axis with a Neumann wall needs n[d] >= 3");
            }
        }
        total *= g->n[k];
    }
    if (neumann && d && d->ts == EW_TS_IMPLICIT &&
        (d->predictor == EW_PRED_CNN || d->predictor == EW_PRED_PROJ))
        return fail(EW_ERR_UNSUPPORTED, "with Neumann walls the implicit guesses are ZERO, SCALED or EXTRAP "
                                        "(the projection and the network assume a symmetric M)");
    if (total > (int64_t)1 << 34) return fail(EW_ERR_INVALID_ARG, "grid too large");
    if (!(d->omega > 0.0) || !std::isfinite(d->omega)) return fail(EW_ERR_INVALID_ARG, "omega must be > 0");
    if (d->ts != EW_TS_EXPLICIT && d->ts != EW_TS_IMPLICIT) return fail(EW_ERR_INVALID_ARG, "ts must be explicit or implicit");
    if (d->n_p < 1) return fail(EW_ERR_INVALID_ARG, "n_p must be >= 1");
    if (d->filter_const != EW_FILTER_ALPHA_D && d->filter_const != EW_FILTER_QUARTER)
        return fail(EW_ERR_INVALID_ARG, "filter_const must be ALPHA_D or QUARTER");
    if (d->precision != EW_PREC_FP64 && d->precision != EW_PREC_MIXED)
        return fail(EW_ERR_INVALID_ARG, "precision must be FP64 or MIXED");
    if (d->ts == EW_TS_EXPLICIT) {
        if (!(d->cfl > 0.0 && d->cfl <= 1.0)) return fail(EW_ERR_INVALID_ARG, "cfl must be in (0, 1]");
        if (d->adjust_omega) return fail(EW_ERR_INVALID_ARG, "adjust_omega applies to implicit stepping only");
    } else {
        if (d->n_its < 5) return fail(EW_ERR_INVALID_ARG, "n_its must be >= 5");
        if (!(d->mg_tol > 0.0 && d->mg_tol < 1.0)) return fail(EW_ERR_INVALID_ARG, "mg_tol must be in (0, 1)");
        if (d->mg_nu1 < 0 || d->mg_nu2 < 0 || d->mg_nu1 + d->mg_nu2 < 1 || d->mg_nu1 > 8 || d->mg_nu2 > 8)
            return fail(EW_ERR_INVALID_ARG, "mg_nu1, mg_nu2 must be in [0, 8] with nu1 + nu2 >= 1");
        if (d->mg_max_cycles < 1 || d->mg_max_cycles > 10000) return fail(EW_ERR_INVALID_ARG, "mg_max_cycles must be in [1, 10000]");
        if (d->mg_coarse_sweeps < 1 || d->mg_coarse_sweeps > 10000)
            return fail(EW_ERR_INVALID_ARG, "mg_coarse_sweeps must be in [1, 10000]");
        if (d->mg_coarse_points < 0) return fail(EW_ERR_INVALID_ARG, "mg_coarse_points must be >= 0");
        if (d->predictor != EW_PRED_ZERO && d->predictor != EW_PRED_SCALED && d->predictor != EW_PRED_CNN &&
            d->predictor != EW_PRED_EXTRAP && d->predictor != EW_PRED_PROJ)
            return fail(EW_ERR_INVALID_ARG, "unknown predictor");
        if (d->proj_window > 32) return fail(EW_ERR_INVALID_ARG, "proj_window must be at most 32");
        if (d->mg_max_levels < EW_MG_LEVELS_AUTO)
            return fail(EW_ERR_INVALID_ARG, "mg_max_levels must be >= 0 or EW_MG_LEVELS_AUTO");
        if (!(d->mg_relax == 0.0 || (d->mg_relax > 0.0 && d->mg_relax < 2.0)))
            return fail(EW_ERR_INVALID_ARG, "mg_relax must be 0 (default) or in (0, 2)");
        if (!(d->mg_relax_coarse == 0.0 || (d->mg_relax_coarse > 0.0 && d->mg_relax_coarse < 2.0)))
            return fail(EW_ERR_INVALID_ARG, "mg_relax_coarse must be 0 (default) or in (0, 2)");
        if (d->predictor == EW_PRED_CNN && (g->dim != 2))
            return fail(EW_ERR_UNSUPPORTED, "the learned predictor is implemented for 2D grids");
    }
    return EW_OK;
}

ew_status Op::build_hierarchy() {
    // Level sizes: halve (n-1)/2 while every n_d is odd and >= 3.
    std::vector<std::array<int64_t, 3>> sizes;
    std::array<int64_t, 3> cur = {n[0], n[1], dim == 3 ? n[2] : 1};
    sizes.push_back(cur);
    const size_t max_levels = desc.mg_max_levels > 0 ? (size_t)desc.mg_max_levels : 64;
    // EW_MG_LEVELS_AUTO: level l (spacings h 2^l) ends the hierarchy once
    // mg_coarse_sweeps Gauss-Seidel sweeps contract it by 0.1 (Gershgorin
    // bound of the Jacobi radius, squared for red-black Gauss-Seidel).
    auto coarse_enough = [&](size_t l) -> bool {
        double s = 0.0;
        for (int k = 0; k < dim; ++k) {
            const double hl = h[k] * std::ldexp(1.0, (int)l);
            s += 1.0 / (hl * hl);
        }
        const double off = (order == 2 ? 2.0 : 34.0 / 12.0) * a * s;
        const double diag = 1.0 + (order == 2 ? 2.0 : 30.0 / 12.0) * a * s;
        const double rho_gs = (off / diag) * (off / diag);
        return off < diag && std::pow(rho_gs, desc.mg_coarse_sweeps) <= 0.1;
    };
    // Coarsening per axis keeps the walls' points: Dirichlet-Dirichlet n = 2 n_c
    // + 1; one Neumann wall n = 2 n_c (the wall point is a coarse point);
    // Neumann-Neumann n = 2 n_c - 1.  An axis with a Neumann wall keeps at
    // least 3 points.
    auto coarsen = [&](int k, int64_t m, int64_t* mc) -> bool {
        const int nn = ((g.wall >> (2 * k)) & 1) + ((g.wall >> (2 * k + 1)) & 1);
        if (nn == 0) {
            if (m % 2 != 1 || m < 3) return false;
            *mc = (m - 1) / 2;
            return true;
        }
        const int64_t c = nn == 1 ? (m % 2 == 0 ? m / 2 : -1) : (m % 2 == 1 ? (m + 1) / 2 : -1);
        if (c < 3 || c >= m) return false;
        *mc = c;
        return true;
    };
    while (sizes.size() < max_levels) {
        if (desc.mg_max_levels == EW_MG_LEVELS_AUTO && coarse_enough(sizes.size() - 1)) break;
        std::array<int64_t, 3> nxt = cur;
        bool ok = true;
        for (int k = 0; k < dim; ++k) ok = ok && coarsen(k, cur[k], &nxt[k]);
        if (!ok) break;
        cur = nxt;
        sizes.push_back(cur);
    }
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    levels.resize(sizes.size());
    for (size_t l = 0; l < sizes.size(); ++l) {
        Level& L = levels[l];
        double hl[3];
        for (int k = 0; k < 3; ++k) hl[k] = h[k] * std::ldexp(1.0, (int)l);
        L.g = make_geo(dim, sizes[l].data(), hl, g.wall);
        const int64_t m = L.g.size();
        // Level 0 of the FP64 solver works on the caller's x with one partner
        // buffer; every other level (and every level of the FP32 inner solver)
        // owns x, its partner and b.
        EW_TRY(alloc(&L.x[1], m * es));
        if (l > 0 || mixed) {
            EW_TRY(alloc(&L.x[0], m * es));
            EW_TRY(alloc(&L.b, m * es));
        }
    }
    // Levels from coarse_level down run in one workgroup with x and b of every
    // such level resident in LDS.
    const int nlev = (int)levels.size();
    coarse_level = nlev;
    if (g.wall) return EW_OK;  // the one-workgroup kernel has the Dirichlet closure only: tiles on every level
    const int64_t cap_pts = desc.mg_coarse_points > 0 ? desc.mg_coarse_points : (int64_t)1 << 40;
    auto padded = [&](const Geo& gq) -> int64_t {
        return (int64_t)(gq.nx + 4) * (gq.ny + 4) * (dim == 3 ? gq.nz + 4 : 1);
    };
    for (int l = nlev - 1; l >= 0; --l) {
        const Geo& gl = levels[l].g;
        const int64_t m = gl.size();
        const int cap = dim == 2 ? kCoarseMax2D : kCoarseMax3D;
        if (gl.nx > cap || gl.ny > cap || (dim == 3 && gl.nz > cap) || m > cap_pts) break;
        if (nlev - l > kMaxCoarseLevels) break;
        int64_t elems = (padded(gl) + 1) & ~(int64_t)1;  // residual scratch
        for (int q = l; q < nlev; ++q) elems += (2 * padded(levels[q].g) + 1) & ~(int64_t)1;
        if (elems * (int64_t)es > (int64_t)kCoarseMaxLdsBytes) break;
        coarse_level = l;
    }
    if (coarse_level < nlev) {
        coarse.nlev = nlev - coarse_level;
        int off = 0;
        for (int q = 0; q < coarse.nlev; ++q) {
            const Geo& gq = levels[coarse_level + q].g;
            coarse.g[q] = gq;
            coarse.off_x[q] = off;
            off += (int)padded(gq);
            coarse.off_b[q] = off;
            off += (int)padded(gq);
            off = (off + 1) & ~1;  // keep 16-byte alignment for FP32 pairs
        }
        coarse.off_r = off;
        off += (int)padded(coarse.g[0]);
        off = (off + 1) & ~1;
        coarse.lds_elems = off;
        // The attribute is per kernel, not per operator: always allow the maximum.
        hipError_t e = mixed ? prepare_coarse_vcycle<float>(dim, order, kCoarseMaxLdsBytes)
                             : prepare_coarse_vcycle<double>(dim, order, kCoarseMaxLdsBytes);
        if (e != hipSuccess) return fail(EW_ERR_HIP, std::string("coarse kernel LDS: ") + hipGetErrorString(e));
    }
    return EW_OK;
}

}  // namespace ew

using namespace ew;

namespace ew {
void grid_geometry(const ew_grid_desc* grid, int64_t n[3], double len[3], double h[3], int* wall) {
    *wall = 0;
    for (int k = 0; k < 3; ++k) {
        n[k] = k < grid->dim ? grid->n[k] : 1;
        len[k] = k < grid->dim ? grid->len[k] : 1.0;
        int nn = 0;
        for (int e = 0; e < 2 && k < grid->dim; ++e)
            if (grid->walls[k][e] == EW_WALL_NEUMANN) {
                *wall |= 1 << (2 * k + e);
                ++nn;
            }
        // a Neumann wall point is active: h = len / (n + 1 - Neumann walls)
        h[k] = len[k] / (double)(n[k] + 1 - nn);
    }
}

// Default relaxation weights of the box smoothers: 1.2 on the finest level,
// 1.05 on the coarser ones.  Measured in the V-cycles per implicit solve of
// an Arnoldi sequence (one weight on every level before): the 2047^2 order-4
// headline 9.56 (1.1 everywhere) -> 8.99; 1023^2 order 4 at omega 90, 9.72 ->
// 8.93; 2047^2 order 2 at omega 60, 8.86 -> 8.43; the 255^3 mixed cube, 9.2
// (1.15 everywhere) -> 8.4; the 127^3 cube unchanged.  The finest level, where
// a dt^2 / h^2 is largest, wants the most over-relaxation.
double default_relax(double mg_relax, int dim, int order) {
    (void)dim;
    (void)order;
    return mg_relax != 0.0 ? mg_relax : 1.2;
}
}  // namespace ew

extern "C" ew_status ew_op_create(const ew_grid_desc* grid, const ew_op_desc* desc, void* hip_stream, ew_op* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    EW_TRY(validate_descs(grid, desc));
    std::unique_ptr<ew_op_s> op(new ew_op_s());
    op->dim = grid->dim;
    op->order = grid->order;
    int wall = 0;
    grid_geometry(grid, op->n, op->len, op->h, &wall);
    op->desc = *desc;
    op->stream = (hipStream_t)hip_stream;
    op->mixed = desc->precision == EW_PREC_MIXED;
    op->implicit = desc->ts == EW_TS_IMPLICIT;
    op->g = make_geo(op->dim, op->n, op->h, wall);
    op->N = op->g.size();
    EW_HIP_TRY(hipGetDevice(&op->device));
    make_plan(op.get());
    op->a = 0.5 * op->dt * op->dt;
    op->relax = default_relax(desc->mg_relax, op->dim, op->order);
    op->relax_coarse = desc->mg_relax_coarse != 0.0 ? desc->mg_relax_coarse : kDefaultRelaxCoarse;

    const int64_t N = op->N;
    EW_TRY(op->alloc((void**)&op->partial_dev, kRedBlocks * sizeof(double) * 4));
    EW_HIP_TRY(hipHostMalloc((void**)&op->partial_host, kRedBlocks * sizeof(double) * 4, hipHostMallocDefault));
    EW_TRY(op->alloc((void**)&op->wA, N * sizeof(double)));
    EW_TRY(op->alloc((void**)&op->wB, N * sizeof(double)));
    if (op->implicit) {
        EW_TRY(op->alloc((void**)&op->sbuf, N * sizeof(double)));
        EW_TRY(op->alloc((void**)&op->tile_partial_dev, residual_tiles(op->g) * sizeof(double)));
        EW_TRY(op->build_hierarchy());
        EW_TRY(op->proj_setup());
        if (op->mixed) {
            EW_TRY(op->alloc((void**)&op->acc32, N * sizeof(float)));
        }
    } else {
        EW_TRY(op->alloc((void**)&op->c_dev, op->c.size() * sizeof(double)));
        EW_HIP_TRY(hipMemcpy(op->c_dev, op->c.data(), op->c.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!op->implicit && op->mixed) {
        EW_TRY(op->alloc((void**)&op->f0, N * sizeof(float)));
        EW_TRY(op->alloc((void**)&op->fA, N * sizeof(float)));
        EW_TRY(op->alloc((void**)&op->fB, N * sizeof(float)));
        EW_TRY(op->alloc((void**)&op->acc32, N * sizeof(float)));
    }
    *out = op.release();
    return EW_OK;
}

extern "C" void ew_op_destroy(ew_op op) { delete op; }

extern "C" ew_status ew_set_allocator(ew_alloc_fn alloc, ew_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(EW_ERR_INVALID_ARG, "ew_set_allocator needs both functions or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    const int64_t live = g_live_blocks.load();
    if (live != 0)
        return fail(EW_ERR_INVALID_ARG, std::to_string(live) + " library buffers are live; destroy every operator, "
                                        "batch and network first");
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_ctx = ctx;
    return EW_OK;
}

extern "C" ew_status ew_op_get_info(ew_op op, ew_op_info* out) {
    if (!op || !out) return fail(EW_ERR_INVALID_ARG, "null argument");
    out->n_active = op->N;
    out->n_t = op->n_t;
    out->dt = op->dt;
    out->omega_used = op->omega_used;
    out->t_final = op->t_final;
    out->alpha_d = op->alpha_d;
    out->mg_levels = (int)op->levels.size();
    out->mg_relax = op->relax;
    out->mg_relax_coarse = op->relax_coarse;
    return EW_OK;
}

extern "C" ew_status ew_op_get_stats(ew_op op, ew_op_stats* out) {
    if (!op || !out) return fail(EW_ERR_INVALID_ARG, "null argument");
    *out = op->stats;
    return EW_OK;
}

extern "C" ew_status ew_op_probe_guesses(ew_op op, int on) {
    if (!op) return fail(EW_ERR_INVALID_ARG, "null op");
    if (!op->implicit || op->mixed || op->mapped)
        return fail(EW_ERR_INVALID_ARG, "guess probes need an implicit FP64 box operator");
    op->probe_guess = on != 0;
    return EW_OK;
}

extern "C" ew_status ew_op_reset_stats(ew_op op) {
    if (!op) return fail(EW_ERR_INVALID_ARG, "null op");
    std::memset(&op->stats, 0, sizeof(op->stats));
    return EW_OK;
}

extern "C" ew_status ew_op_apply_laplacian(ew_op op, const double* v_dev, double* out_dev) {
    if (!op || !v_dev || !out_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (v_dev == out_dev) return fail(EW_ERR_INVALID_ARG, "v and out may not alias");
    if (op->mapped) EW_HIP_TRY(launch_laplacian_mapped(v_dev, out_dev, op->g, op->mc, op->stream));
    else EW_HIP_TRY(launch_laplacian<double>(v_dev, out_dev, op->g, op->order, op->stream));
    op->stats.laplacian_applies++;
    return EW_OK;
}

extern "C" ew_status ew_op_profile_begin(ew_op op, int kclass, int level) {
    if (!op) return fail(EW_ERR_INVALID_ARG, "null op");
    if (kclass < EW_K_LEAPFROG || kclass > EW_K_SMOOTH_ZERO) return fail(EW_ERR_INVALID_ARG, "unknown kernel class");
    op->prof.kclass = kclass;
    op->prof.level = level;
    op->prof.used = 0;
    op->prof.launches = 0;
    op->prof.bytes = 0.0;
    return EW_OK;
}

extern "C" ew_status ew_op_profile_end(ew_op op, ew_kernel_profile* out) {
    if (!op || !out) return fail(EW_ERR_INVALID_ARG, "null argument");
    Profiler& p = op->prof;
    double total = 0.0;
    if (p.used > 0) EW_HIP_TRY(hipEventSynchronize(p.pool[p.used - 1]));
    for (size_t i = 0; i + 1 < p.used; i += 2) {
        float ms = 0.0f;
        EW_HIP_TRY(hipEventElapsedTime(&ms, p.pool[i], p.pool[i + 1]));
        total += ms;
    }
    out->launches = p.launches;
    out->total_ms = total;
    out->bytes_alg = p.bytes;
    p.kclass = -1;
    p.used = 0;
    return EW_OK;
}
