// The operator object behind ew_op.
#pragma once

#include <array>
#include <functional>
#include <string>
#include <vector>

#include "ew_internal.h"
#include "mg_tile.h"

namespace ew {

// One multigrid level.  Storage type is double for the FP64 solver and float
// for the FP32 inner solver of the mixed-precision defect correction.
struct Level {
    Geo g;
    void* x[2] = {nullptr, nullptr};  // iterate and its out-of-place partner
    void* b = nullptr;                // right-hand side (restricted residual)
};

struct Cnn;  // learned warm start (cnn.hip)

constexpr int kProjMax = 32;     // largest projection window
constexpr int kProjBlocks = 1024; // reduction blocks of the projection kernels

// hipEvent timing of one kernel class (ew_op_profile_*).
struct Profiler {
    int kclass = -1, level = -1;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int64_t launches = 0;
    double bytes = 0.0;
    static constexpr size_t kMaxLaunches = 65536;
    bool wants(int kc, int lv) const { return kc == kclass && (level < 0 || level == lv) && used + 2 <= 2 * kMaxLaunches; }
};

// Time step, step count and filter weights of one wave-solve (computed in
// FP64 on the host, in the order of operations of the definition).
struct TimePlan {
    double omega_used = 0, t_final = 0, dt = 0, alpha_d = 0;
    double shift = 0;          // the filter constant: alpha_d / 2 or 1/4
    int n_t = 0;
    std::vector<double> c;
};
// rho_override > 0 replaces the box bound sum_d c / h_d^2 on the spectrum of
// -L_h in the explicit time step (a mapped grid supplies its own).  With
// with_weights = false the weights c_k are left out (filter_weight gives each).
void make_time_plan(int dim, int order, const double* h, const ew_op_desc& d, TimePlan& tp,
                    double rho_override = 0.0, bool with_weights = true);
double filter_weight(const TimePlan& tp, int k);
// Active-point counts, spacings and Neumann-wall bits of a validated grid
// descriptor (h = len / (n + 1 - Neumann walls of the axis)).
void grid_geometry(const ew_grid_desc* grid, int64_t n[3], double len[3], double h[3], int* wall);
ew_status validate_descs(const ew_grid_desc* g, const ew_op_desc* d);
double default_relax(double mg_relax, int dim, int order);
constexpr double kDefaultRelaxCoarse = 1.05;  // weight of the coarser levels' box smoothers

// Whole explicit wave-solve of a small 2D grid in one workgroup (wave_small.hip).
template <typename T>
bool wave_small_fits(const Geo& g);
template <typename T>
hipError_t launch_wave_small(const double* v, double* out, const Geo& g, int order, double dt2, const double* c_dev,
                             int n_t, hipStream_t s);

struct Op;
// Brackets one launch with events when the profiler asks for it.
struct ProfScope {
    Op* op;
    bool on;
    bool external;  // the launch records the events itself (start_event/stop_event)
    ProfScope(Op* o, int kclass, int level, double bytes, bool external_events = false);
    ~ProfScope();
    hipEvent_t start_event() const;
    hipEvent_t stop_event() const;
};

struct Op {
    // grid
    int dim = 2, order = 2;
    int64_t n[3] = {1, 1, 1};
    double len[3] = {1, 1, 1}, h[3] = {1, 1, 1};
    Geo g{};
    int64_t N = 0;
    // operator
    ew_op_desc desc{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool mixed = false, implicit = false;
    double omega_used = 0, t_final = 0, dt = 0, alpha_d = 0, a = 0;
    double relax = 1.0;         // relaxation weight of the finest level's box smoother (resolved mg_relax)
    double relax_coarse = 1.0;  // ... of the coarser levels (resolved mg_relax_coarse)
    int n_t = 0;
    std::vector<double> c;
    // single curvilinear grid (explicit FP64 only): coefficients of the mapped operator
    bool mapped = false;
    MapCoef mc{};
    double map_rho = 0.0;      // Gershgorin bound on the spectrum of -L_h
    std::vector<MapCoef> mcoef;  // per multigrid level (implicit)
    // workspace
    double* wA = nullptr;
    double* wB = nullptr;
    double* wC = nullptr;  // second state pair of the blocked explicit steps (allocated at first use)
    double* wD = nullptr;
    double* sbuf = nullptr;
    float* f0 = nullptr;
    float* fA = nullptr;
    float* fB = nullptr;
    float* acc32 = nullptr;
    double* c_dev = nullptr;   // filter weights c_0..c_{N_t} on the device (explicit operators)
    double* partial_dev = nullptr;
    double* partial_host = nullptr;
    double* tile_partial_dev = nullptr;  // per-tile residual sums of the finest level (implicit boxes)
    std::vector<Level> levels;
    int coarse_level = 0;      // first level run by the single-workgroup kernel
    CoarseLevels coarse{};
    // Speculative residual tests, kept per kind of solve (0: the first step's
    // M W^1 = W^0 of a wave-solve, 1: the steps M S = 2 W^n, whose guesses
    // differ): V-cycles of the previous solve of that kind, and whether it met
    // the tolerance at its first test (then it may have run more cycles than it
    // needed, and the next solve of the kind tests one cycle earlier).
    int spec_cycles[2] = {0, 0};
    bool spec_first_pass[2] = {false, false};
    int solve_kind = 1;        // kind of the solve in progress
    std::vector<void*> allocations;
    Cnn* cnn = nullptr;
    // ||b||^2 already known for the right-hand side b_src of the next solve
    // (the learned guess computes it); consumed by that solve.
    const double* bb_src = nullptr;
    double bb_val = 0.0;
    // Called at every implicit solve M x = bscale b of a step n >= 1 once the
    // base guess x0 is formed, before the multigrid, with (b, bscale, x0,
    // x0 taken as zero and not yet written); used to record training crops.
    std::function<ew_status(const double*, double, double*, bool)> guess_hook;
    double* cnn_r = nullptr;   // residual of the base guess (learned correction)
    bool probe_guess = false;  // measure the initial residuals (ew_op_probe_guesses)
    // Projection guess (proj.hip): FP32 copies of the last proj_k solutions
    // in a ring of slots, and their Gram matrix G[s][t] = x_s . b_t on the
    // host (row-major, kProjMax x kProjMax).
    int proj_k = 0;            // window size (0 = projection off)
    int proj_count = 0;        // filled slots
    int proj_head = 0;         // slot the next pair goes to
    bool proj_pending = false; // Gram row of the last added pair still on the device
    int proj_pending_slot = -1;
    bool proj_rhs_ok = false;  // proj_c holds the products for the solve in progress
    float* proj_X = nullptr;       // proj_k rows of proj_ld floats
    int64_t proj_ld = 0;
    double* proj_partial = nullptr;  // kProjBlocks x (kProjMax + 1) per result set
    double* proj_res_dev = nullptr;  // 2 x (kProjMax + 1): products with b, Gram row of the last pair
    double* proj_res_host = nullptr;
    std::vector<double> proj_G;
    std::vector<double> proj_c;   // x_v . (bscale b) for the solve in progress
    int64_t proj_guesses = 0;
    ew_op_stats stats{};
    Profiler prof;

    ~Op();
    ew_status alloc(void** p, size_t bytes);
    ew_status host_sum_partials(double* out);
    ew_status build_hierarchy();

    // multigrid (wave.hip)
    // Relaxation weight of level l: 1 on a single-point level, where one
    // half-sweep with weight 1 is the exact solve.
    double level_relax(int l) const {
        return levels[l].g.size() == 1 ? 1.0 : (l == 0 ? relax : relax_coarse);
    }
    template <typename T>
    ew_status vcycle(int level, T* cur, T* other, const T* b, double bscale, bool zero, T** result);
    template <typename T>
    ew_status sweep(int level, T*& cur, T*& other, const T* b, double bscale, bool zero, const T* xc);
    template <typename T>
    ew_status sweeps(int level, int count, T*& cur, T*& other, const T* b, double bscale, bool zero);
    ew_status mapped_vcycle(int level, double* cur, double* other, const double* b, double bscale, bool zero,
                            double** result);
    ew_status mg_solve64(const double* b, double bscale, double* x, bool x_is_zero, int* cycles, double* rel,
                         bool speculate = false);
    ew_status mg_solve_mixed(const double* b, double bscale, double* x, bool x_is_zero, int* cycles, double* rel,
                             bool speculate = false);
    ew_status rhs_norm2(const double* b, double* bb);
    ew_status proj_setup();
    ew_status proj_guess(const double* b, double bscale, double* x, bool* x_is_zero);
    ew_status proj_add(const double* b, double bscale, const double* x);
    ew_status implicit_solve(const double* b, double bscale, double* x, const double* wprev_for_guess);
    ew_status guess_rel_res(const double* b, double bscale, const double* x, double* rel);
    ew_status apply_filter(const double* v, double* out);
};

}  // namespace ew

struct ew_op_s : public ew::Op {};
