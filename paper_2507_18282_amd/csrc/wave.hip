// The wave-solve with time filter (S v) and the implicit step's multigrid
// solver, orchestrated on the host and executed by the kernels of
// stencil.hip and mg.hip on the operator's stream.
#include <algorithm>
#include <cmath>

#include "op.h"

namespace ew {

// One full red-black sweep on level l, out of place: cur -> other, then the
// two pointers swap so that cur holds the result.  With xc != nullptr the
// prolongation of xc (level l+1) is added to the iterate first; with zero the
// incoming iterate is taken as zero without being read.
template <typename T>
ew_status Op::sweep(int l, T*& cur, T*& other, const T* b, double bscale, bool zero, const T* xc) {
    const Level& L = levels[l];
    const Geo gc = (xc != nullptr) ? levels[l + 1].g : L.g;
    const double n = (double)L.g.size();
    const double w = level_relax(l);
    double bytes = sizeof(T) * ((zero ? 2.0 : 3.0) * n);
    if (xc) bytes += sizeof(T) * (double)gc.size();
    {
        ProfScope ps(this, xc ? EW_K_PROLONG : (zero ? EW_K_SMOOTH_ZERO : EW_K_SMOOTH), l, bytes, true);
        EW_HIP_TRY(launch_sweep_tile<T>(cur, xc, b, bscale, other, L.g, gc, order, a, w, zero, xc != nullptr, stream,
                                        ps.start_event(), ps.stop_event()));
    }
    std::swap(cur, other);
    return EW_OK;
}

// `count` consecutive plain sweeps on level l (the first from zero if `zero`):
// on 2D levels pairs of sweeps run as one fused pass.
template <typename T>
ew_status Op::sweeps(int l, int count, T*& cur, T*& other, const T* b, double bscale, bool zero) {
    const Level& L = levels[l];
    const double n = (double)L.g.size();
    int s = 0;
    if (L.g.dim == 2) {
        for (; s + 1 < count; s += 2) {
            const bool z = zero && s == 0;
            // algorithmic bytes counted per sweep (x, b read and x written once per
            // sweep), for the two sweeps this launch performs
            ProfScope ps(this, z ? EW_K_SMOOTH_ZERO : EW_K_SMOOTH, l, sizeof(T) * ((z ? 5.0 : 6.0) * n), true);
            EW_HIP_TRY(launch_sweep2x2d<T>(cur, b, bscale, other, L.g, order, a, level_relax(l), z, stream,
                                           ps.start_event(),
                                           ps.stop_event()));
            std::swap(cur, other);
        }
    }
    for (; s < count; ++s) EW_TRY(sweep<T>(l, cur, other, b, bscale, zero && s == 0, nullptr));
    return EW_OK;
}

// V(nu1, nu2) cycle on level l starting from the iterate in cur (zero if
// `zero`); other is its partner buffer.  *result receives the buffer that holds
// the new iterate (cur or other).  Levels from coarse_level down run in one
// workgroup; a coarsest level of one point is solved exactly and a larger one
// gets mg_coarse_sweeps sweeps.
template <typename T>
ew_status Op::vcycle(int l, T* cur, T* other, const T* b, double bscale, bool zero, T** result) {
    const int last = (int)levels.size() - 1;
    const Level& L = levels[l];
    if (l >= coarse_level) {
        // the coarse range must start at this level
        CoarseLevels c = coarse;
        {
            ProfScope ps(this, EW_K_COARSE, l, sizeof(T) * 3.0 * (double)L.g.size());
            EW_HIP_TRY(launch_coarse_vcycle<T>(b, bscale, zero ? nullptr : cur, cur, c, order, a, level_relax(l),
                                               relax_coarse, desc.mg_nu1, desc.mg_nu2, desc.mg_coarse_sweeps,
                                               stream));
        }
        *result = cur;
        return EW_OK;
    }
    if (l == last) {
        EW_TRY(sweeps<T>(l, L.g.size() == 1 ? 1 : desc.mg_coarse_sweeps, cur, other, b, bscale, zero));
        *result = cur;
        return EW_OK;
    }
    const Level& C = levels[l + 1];
    // 2D levels below 1024 tiles of 64 x 16 (511^2 and smaller here) without
    // Neumann walls: the last two pre-smoothing sweeps, the residual and its
    // restriction in one pass, which saves a launch where launches, not bytes,
    // set the time.  On larger levels the wider relaxed region it needs costs
    // more than the separate restriction pass (2047^2: 64.0 us against 36.3 +
    // 16.3; 1023^2: 18.5 against 11.8 + 5.9; 511^2: 9.6 against 6.0 + 4.6).
    const bool small2d = L.g.dim == 2 && (int64_t)((L.g.nx + 63) / 64) * ((L.g.ny + 15) / 16) < 1024;
    if (small2d && !L.g.wall && desc.mg_nu1 >= 2 && desc.mg_nu1 % 2 == 0) {
        EW_TRY(sweeps<T>(l, desc.mg_nu1 - 2, cur, other, b, bscale, zero));
        const bool z = zero && desc.mg_nu1 == 2;
        const double n = (double)L.g.size();
        // algorithmic bytes: two sweeps (x, b read and x written per sweep) and
        // the restriction (x, b read, coarse b written)
        ProfScope ps(this, z ? EW_K_SMOOTH_ZERO : EW_K_SMOOTH, l,
                     sizeof(T) * ((z ? 5.0 : 6.0) * n + 2.0 * n + (double)C.g.size()), true);
        EW_HIP_TRY(launch_sweep2x_restrict2d<T>(cur, b, bscale, other, L.g, order, a, level_relax(l), z, (T*)C.b,
                                                C.g, stream, ps.start_event(), ps.stop_event()));
        std::swap(cur, other);
    } else {
        EW_TRY(sweeps<T>(l, desc.mg_nu1, cur, other, b, bscale, zero));
        if (desc.mg_nu1 == 0 && zero) EW_HIP_TRY(launch_fill<T>(cur, L.g.size(), T(0), stream));
        ProfScope ps(this, EW_K_RESTRICT, l, sizeof(T) * (2.0 * L.g.size() + C.g.size()));
        EW_HIP_TRY(launch_restrict_tile<T>(cur, b, bscale, L.g, order, a, (T*)C.b, C.g, stream));
    }
    T* xc = nullptr;
    EW_TRY(vcycle<T>(l + 1, (T*)C.x[0], (T*)C.x[1], (T*)C.b, 1.0, true, &xc));
    if (desc.mg_nu2 >= 1 && L.g.dim == 3 && !sweep_z3d_fuses_prolong(L.g, order)) {
        // 3D: the prolongation as its own pass (interpolating inside the staged
        // sweep tile reads each coarse value up to eight times from the cache)
        {
            ProfScope ps(this, EW_K_PROLONG, l, sizeof(T) * (2.0 * L.g.size() + C.g.size()));
            EW_HIP_TRY(launch_prolong_correct<T>(cur, xc, L.g, C.g, stream));
        }
        for (int s = 0; s < desc.mg_nu2; ++s) EW_TRY(sweep<T>(l, cur, other, b, bscale, false, nullptr));
    } else if (desc.mg_nu2 >= 1) {
        EW_TRY(sweep<T>(l, cur, other, b, bscale, false, xc));
        for (int s = 1; s < desc.mg_nu2; ++s) EW_TRY(sweep<T>(l, cur, other, b, bscale, false, nullptr));
    } else {
        ProfScope ps(this, EW_K_PROLONG, l, sizeof(T) * (2.0 * L.g.size() + C.g.size()));
        EW_HIP_TRY(launch_prolong_correct<T>(cur, xc, L.g, C.g, stream));
    }
    *result = cur;
    return EW_OK;
}

static ew_status check_rel(double rel) {
    if (!std::isfinite(rel)) return fail(EW_ERR_NONFINITE, "non-finite multigrid residual");
    return EW_OK;
}

// FP64 multigrid: x <- M^{-1} (bscale b) to ||r||_2 <= mg_tol ||bscale b||_2.
// With `speculate`, the first cycles run without the residual test, which
// costs a pass over x and b and a host round trip: as many as the previous
// solve of the same kind took minus one (minus two if that solve met the
// tolerance at its first test, so that a falling count is followed); the test
// then runs after every further cycle, so the solve still stops at the first
// tested cycle that meets the tolerance.
ew_status Op::rhs_norm2(const double* b, double* bb) {
    if (bb_src == b) {
        *bb = bb_val;
        bb_src = nullptr;
        return EW_OK;
    }
    bb_src = nullptr;
    EW_HIP_TRY(launch_dot_partial(b, b, N, partial_dev, stream));
    return host_sum_partials(bb);
}

ew_status Op::mg_solve64(const double* b, double bscale, double* x, bool x_is_zero, int* cycles, double* rel_out,
                         bool speculate) {
    double bb = 0.0;
    EW_TRY(rhs_norm2(b, &bb));
    const double bn = std::sqrt(bb) * std::fabs(bscale);
    if (!std::isfinite(bn)) return fail(EW_ERR_NONFINITE, "non-finite right-hand side");
    int cyc = 0;
    double rel = 0.0;
    if (bn == 0.0) {
        EW_HIP_TRY(launch_fill<double>(x, N, 0.0, stream));
    } else {
        const int kind = solve_kind;
        const int skip = speculate && spec_cycles[kind] > 0
                             ? std::max(0, spec_cycles[kind] - (spec_first_pass[kind] ? 2 : 1))
                             : 0;
        int tests = 0;
        double* cur = x;
        double* other = (double*)levels[0].x[1];
        bool zero = x_is_zero;
        for (;;) {
            const bool test = cyc >= skip && !(zero && cyc == 0);
            if (test) {
                {
                    ProfScope ps(this, EW_K_RESNORM, 0, 16.0 * (double)N);
                    if (mapped)
                        EW_HIP_TRY(launch_residual_mapped(cur, b, bscale, g, mcoef[0], a, partial_dev, nullptr, stream));
                    else
                        EW_HIP_TRY((launch_residual_tile<double, double>(cur, b, bscale, g, order, a, tile_partial_dev,
                                                                         partial_dev, nullptr, stream)));
                }
                double rr;
                EW_TRY(host_sum_partials(&rr));
                rel = std::sqrt(rr) / bn;
                EW_TRY(check_rel(rel));
                ++tests;
                if (rel <= desc.mg_tol) break;
            } else {
                rel = 1.0;
            }
            if (cyc >= desc.mg_max_cycles) break;
            double* res = nullptr;
            if (mapped) EW_TRY(mapped_vcycle(0, cur, other, b, bscale, zero, &res));
            else EW_TRY(vcycle<double>(0, cur, other, b, bscale, zero, &res));
            if (res != cur) std::swap(cur, other);
            zero = false;
            ++cyc;
        }
        if (cur != x) EW_HIP_TRY(hipMemcpyAsync(x, cur, N * sizeof(double), hipMemcpyDeviceToDevice, stream));
        spec_cycles[kind] = cyc;
        spec_first_pass[kind] = tests == 1 && skip > 0;
    }
    stats.mg_solves++;
    stats.mg_cycles += cyc;
    if (cycles) *cycles = cyc;
    if (rel_out) *rel_out = rel;
    if (rel > desc.mg_tol)
        return fail(EW_ERR_MG_NOT_CONVERGED, "multigrid reached mg_max_cycles with relative residual " +
                                                 std::to_string(rel));
    return EW_OK;
}

// Mixed precision: FP64 defect correction around FP32 V-cycles.  Each outer
// iteration forms r = bscale b - M x in FP64 (stored as FP32 for the inner
// solve), stops if ||r|| <= mg_tol ||bscale b||, else solves M e = r with
// kMixedInnerCycles FP32 V-cycles (the first from zero) and updates x += e in
// FP64.  Two inner cycles shrink the residual by about the square of the
// cycle's contraction (some 3e-3, far above the FP32 rounding of r), so the
// FP64 residual and update passes run half as often for about the same
// number of V-cycles.  Cycle counts (tests, speculation, mg_max_cycles) are
// in V-cycles.
constexpr int kMixedInnerCycles = 2;

ew_status Op::mg_solve_mixed(const double* b, double bscale, double* x, bool x_is_zero, int* cycles,
                             double* rel_out, bool speculate) {
    double bb = 0.0;
    EW_TRY(rhs_norm2(b, &bb));
    const double bn = std::sqrt(bb) * std::fabs(bscale);
    if (!std::isfinite(bn)) return fail(EW_ERR_NONFINITE, "non-finite right-hand side");
    if (x_is_zero) EW_HIP_TRY(launch_fill<double>(x, N, 0.0, stream));
    int cyc = 0;
    double rel = 0.0;
    if (bn != 0.0) {
        Level& L0 = levels[0];
        float* r32 = (float*)L0.b;
        float* e32 = (float*)L0.x[0];
        float* t32 = (float*)L0.x[1];
        // speculative tests as in mg_solve64: the residual is formed every
        // iteration (it is the inner solve's right-hand side), its norm read
        // by the host only from the iteration the previous solve suggests
        const int kind = solve_kind;
        const int skip = speculate && spec_cycles[kind] > 0
                             ? std::max(0, spec_cycles[kind] - (spec_first_pass[kind] ? 2 : 1))
                             : 0;
        int tests = 0;
        for (;;) {
            {
                ProfScope ps(this, EW_K_RESNORM, 0, 20.0 * (double)N);
                EW_HIP_TRY((launch_residual_tile<double, float>(x, b, bscale, g, order, a, tile_partial_dev, partial_dev,
                                                                r32, stream)));
            }
            if (cyc >= skip) {
                double rr;
                EW_TRY(host_sum_partials(&rr));
                rel = std::sqrt(rr) / bn;
                EW_TRY(check_rel(rel));
                ++tests;
                if (rel <= desc.mg_tol) break;
            } else {
                rel = 1.0;
            }
            if (cyc >= desc.mg_max_cycles) break;
            const int inner = std::min(kMixedInnerCycles, desc.mg_max_cycles - cyc);
            float* e = e32;
            float* other = t32;
            for (int c = 0; c < inner; ++c) {
                float* res = nullptr;
                EW_TRY(vcycle<float>(0, e, other, r32, 1.0, c == 0, &res));
                if (res != e) std::swap(e, other);
            }
            EW_HIP_TRY((launch_add_inplace<double, float>(x, e, N, stream)));
            cyc += inner;
        }
        spec_cycles[kind] = cyc;
        spec_first_pass[kind] = tests == 1 && skip > 0;
    }
    stats.mg_solves++;
    stats.mg_cycles += cyc;
    if (cycles) *cycles = cyc;
    if (rel_out) *rel_out = rel;
    if (rel > desc.mg_tol)
        return fail(EW_ERR_MG_NOT_CONVERGED, "multigrid reached mg_max_cycles with relative residual " +
                                                 std::to_string(rel));
    return EW_OK;
}

ew_status cnn_correct(Op* op, const double* b, double bscale, double* x);

// One implicit solve M x = bscale b with the operator's initial-guess rule.
// The learned predictor corrects the projection guess (zero while the window
// is empty or off) at the steps n >= 1, whose right-hand sides 2 W^n it was
// trained on; the first step M W^1 = W^0 keeps the projection guess.
ew_status Op::implicit_solve(const double* b, double bscale, double* x, const double* wprev_for_guess) {
    bool zero = false;
    solve_kind = wprev_for_guess == nullptr ? 0 : 1;
    const bool proj = desc.predictor == EW_PRED_PROJ || desc.predictor == EW_PRED_CNN;
    if (proj) {
        EW_TRY(proj_guess(b, bscale, x, &zero));
    } else if (desc.predictor == EW_PRED_ZERO) {
        zero = true;
    } else if (desc.predictor == EW_PRED_EXTRAP) {
        // W^{n+1} ~ 2 W^n - W^{n-1} gives S = W^{n+1} + W^{n-1} ~ 2 W^n (and W^1 ~ W^0).
        EW_HIP_TRY(launch_scale_copy<double>(x, b, N, bscale, stream));
    } else {
        // M phi = (1 + a mu) phi: exact for every mode at mu = omega^2.
        const double s = bscale / (1.0 + a * omega_used * omega_used);
        EW_HIP_TRY(launch_scale_copy<double>(x, b, N, s, stream));
    }
    if (guess_hook && solve_kind == 1) {
        EW_TRY(guess_hook(b, bscale, x, zero));
        zero = false;  // the hook writes a zero guess out
    }
    double base_rel = -1.0;
    if (probe_guess && solve_kind == 1 && !mixed && !mapped) {
        if (zero) EW_HIP_TRY(launch_fill<double>(x, N, 0.0, stream));
        zero = false;
        EW_TRY(guess_rel_res(b, bscale, x, &base_rel));
    }
    if (desc.predictor == EW_PRED_CNN && cnn != nullptr && solve_kind == 1) {
        if (zero) EW_HIP_TRY(launch_fill<double>(x, N, 0.0, stream));
        EW_TRY(cnn_correct(this, b, bscale, x));
        zero = false;
    }
    if (base_rel >= 0.0) {
        double g = base_rel;
        if (desc.predictor == EW_PRED_CNN && cnn != nullptr) EW_TRY(guess_rel_res(b, bscale, x, &g));
        stats.guess_probes++;
        stats.base_rel_res_sum += base_rel;
        stats.guess_rel_res_sum += g;
    }
    if (mixed) EW_TRY(mg_solve_mixed(b, bscale, x, zero, nullptr, nullptr, true));
    else EW_TRY(mg_solve64(b, bscale, x, zero, nullptr, nullptr, true));
    return proj ? proj_add(b, bscale, x) : EW_OK;
}

// ||bscale b - M x||_2 / ||bscale b||_2 (host-blocking); leaves the cached
// ||b||^2 for the solve that follows.
ew_status Op::guess_rel_res(const double* b, double bscale, const double* x, double* rel) {
    double bb;
    if (bb_src == b) {
        bb = bb_val;
    } else {
        EW_HIP_TRY(launch_dot_partial(b, b, N, partial_dev, stream));
        EW_TRY(host_sum_partials(&bb));
        bb_src = b;
        bb_val = bb;
    }
    EW_HIP_TRY((launch_residual_tile<double, double>(x, b, bscale, g, order, a, tile_partial_dev, partial_dev, nullptr,
                                                     stream)));
    double rr;
    EW_TRY(host_sum_partials(&rr));
    *rel = bb > 0.0 ? std::sqrt(rr / bb) / std::fabs(bscale) : 0.0;
    return EW_OK;
}

ew_status Op::apply_filter(const double* v, double* out) {
    const double dt2 = dt * dt;
    if (mapped && !implicit) {
        // several steps per launch; launches alternate between two state pairs
        if (!wC) {
            EW_TRY(alloc((void**)&wC, N * sizeof(double)));
            EW_TRY(alloc((void**)&wD, N * sizeof(double)));
        }
        double* pair[2][2] = {{wA, wB}, {wC, wD}};
        const double* rc = v;
        const double* rp = nullptr;
        const int per = mapped_steps_per_launch();
        for (int k0 = 0, j = 0; k0 < n_t; k0 += per, j ^= 1) {
            const int ns = std::min(per, n_t - k0);
            ProfScope ps(this, EW_K_LEAPFROG, 0, ((k0 == 0 ? 56.0 : 72.0) + 72.0 * (ns - 1)) * (double)N);
            EW_HIP_TRY(launch_leapfrog_mapped_blocked(rc, rp, pair[j][0], pair[j][1], out, g, mc, dt2, c_dev, k0, ns,
                                                      stream));
            rc = pair[j][0];
            rp = pair[j][1];
        }
    } else if (!implicit && (mixed ? wave_small_fits<float>(g) : wave_small_fits<double>(g))) {
        ProfScope ps(this, EW_K_LEAPFROG, 0, 16.0 * (double)N);
        EW_HIP_TRY(mixed ? launch_wave_small<float>(v, out, g, order, dt2, c_dev, n_t, stream)
                         : launch_wave_small<double>(v, out, g, order, dt2, c_dev, n_t, stream));
    } else if (!implicit && !mixed && g.dim == 2) {
        // several steps per launch, as on mapped grids
        if (!wC) {
            EW_TRY(alloc((void**)&wC, N * sizeof(double)));
            EW_TRY(alloc((void**)&wD, N * sizeof(double)));
        }
        double* pair[2][2] = {{wA, wB}, {wC, wD}};
        const double* rc = v;
        const double* rp = nullptr;
        const int per = box_steps_per_launch(order);
        for (int k0 = 0, j = 0; k0 < n_t; k0 += per, j ^= 1) {
            const int ns = std::min(per, n_t - k0);
            ProfScope ps(this, EW_K_LEAPFROG, 0, ((k0 == 0 ? 24.0 : 40.0) + 40.0 * (ns - 1)) * (double)N);
            EW_HIP_TRY(launch_leapfrog_box_blocked(rc, rp, pair[j][0], pair[j][1], out, g, order, dt2, c_dev, k0, ns,
                                                   stream));
            rc = pair[j][0];
            rp = pair[j][1];
        }
    } else if (!implicit && !mixed) {
        {
            ProfScope ps(this, EW_K_LEAPFROG, 0, 24.0 * (double)N);
            EW_HIP_TRY(launch_leapfrog<double>(v, nullptr, wA, out, g, order, dt2, c[0], c[1], 1, stream));
        }
        const double* prev = v;
        double* cur = wA;
        for (int k = 1; k < n_t; ++k) {
            double* next = (prev == v) ? wB : const_cast<double*>(prev);
            ProfScope ps(this, EW_K_LEAPFROG, 0, 40.0 * (double)N);
            EW_HIP_TRY(launch_leapfrog<double>(cur, prev, next, out, g, order, dt2, 0.0, c[k + 1], 0, stream));
            prev = cur;
            cur = next;
        }
    } else if (!implicit && mixed) {
        EW_HIP_TRY((launch_convert<float, double>(f0, v, N, 1.0, stream)));
        {
            ProfScope ps(this, EW_K_LEAPFROG, 0, 12.0 * (double)N);
            EW_HIP_TRY(launch_leapfrog<float>(f0, nullptr, fA, acc32, g, order, dt2, c[0], c[1], 1, stream));
        }
        float* prev = f0;
        float* cur = fA;
        for (int k = 1; k < n_t; ++k) {
            float* next = (prev == f0) ? fB : prev;
            ProfScope ps(this, EW_K_LEAPFROG, 0, 20.0 * (double)N);
            EW_HIP_TRY(launch_leapfrog<float>(cur, prev, next, acc32, g, order, dt2, 0.0, c[k + 1], 0, stream));
            prev = cur;
            cur = next;
        }
        EW_HIP_TRY((launch_convert<double, float>(out, acc32, N, 1.0, stream)));
    } else {
        // Implicit: M W^1 = W^0, then M S = 2 W^n, W^{n+1} = S - W^{n-1}.
        EW_TRY(implicit_solve(v, 1.0, wA, nullptr));
        if (mixed) EW_HIP_TRY((launch_implicit_update<double, float>(wA, v, wA, acc32, N, c[0], c[1], 1, stream)));
        else EW_HIP_TRY((launch_implicit_update<double, double>(wA, v, wA, out, N, c[0], c[1], 1, stream)));
        const double* prev = v;
        double* cur = wA;
        for (int k = 1; k < n_t; ++k) {
            EW_TRY(implicit_solve(cur, 2.0, sbuf, prev));
            double* next = (prev == v) ? wB : const_cast<double*>(prev);
            ProfScope ps(this, EW_K_UPDATE, 0, (mixed ? 32.0 : 40.0) * (double)N);
            if (mixed)
                EW_HIP_TRY((launch_implicit_update<double, float>(sbuf, prev, next, acc32, N, 0.0, c[k + 1], 0, stream)));
            else
                EW_HIP_TRY((launch_implicit_update<double, double>(sbuf, prev, next, out, N, 0.0, c[k + 1], 0, stream)));
            prev = cur;
            cur = next;
        }
        if (mixed) EW_HIP_TRY((launch_convert<double, float>(out, acc32, N, 1.0, stream)));
    }
    stats.wave_solves++;
    stats.time_steps += n_t;
    stats.pt_updates += N * (int64_t)n_t;
    return EW_OK;
}

template ew_status Op::vcycle<double>(int, double*, double*, const double*, double, bool, double**);
template ew_status Op::vcycle<float>(int, float*, float*, const float*, double, bool, float**);

}  // namespace ew

using namespace ew;

extern "C" ew_status ew_op_apply_filter(ew_op op, const double* v_dev, double* out_dev) {
    if (!op || !v_dev || !out_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (v_dev == out_dev) return fail(EW_ERR_INVALID_ARG, "v and out may not alias");
    return op->apply_filter(v_dev, out_dev);
}

extern "C" ew_status ew_op_mg_solve(ew_op op, const double* b_dev, double* x_dev, int* cycles_host,
                                    double* rel_res_host) {
    if (!op || !b_dev || !x_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (!op->implicit) return fail(EW_ERR_INVALID_ARG, "operator is not implicit");
    if (b_dev == x_dev) return fail(EW_ERR_INVALID_ARG, "b and x may not alias");
    ew_status st = op->mixed ? op->mg_solve_mixed(b_dev, 1.0, x_dev, false, cycles_host, rel_res_host)
                             : op->mg_solve64(b_dev, 1.0, x_dev, false, cycles_host, rel_res_host);
    if (st != EW_OK) return st;
    EW_HIP_TRY(hipStreamSynchronize(op->stream));
    return EW_OK;
}

extern "C" ew_status ew_op_mg_vcycle(ew_op op, const double* b_dev, double* x_dev) {
    if (!op || !b_dev || !x_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (!op->implicit || op->mixed) return fail(EW_ERR_INVALID_ARG, "needs an implicit FP64 operator");
    if (b_dev == x_dev) return fail(EW_ERR_INVALID_ARG, "b and x may not alias");
    double* res = nullptr;
    if (op->mapped) EW_TRY(op->mapped_vcycle(0, x_dev, (double*)op->levels[0].x[1], b_dev, 1.0, false, &res));
    else EW_TRY(op->vcycle<double>(0, x_dev, (double*)op->levels[0].x[1], b_dev, 1.0, false, &res));
    if (res != x_dev)
        EW_HIP_TRY(hipMemcpyAsync(x_dev, res, op->N * sizeof(double), hipMemcpyDeviceToDevice, op->stream));
    return EW_OK;
}

extern "C" ew_status ew_op_mg_half_sweep(ew_op op, const double* b_dev, double* x_dev, int colour) {
    if (!op || !b_dev || !x_dev) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (!op->implicit || op->mixed) return fail(EW_ERR_INVALID_ARG, "needs an implicit FP64 operator");
    if (colour != 0 && colour != 1) return fail(EW_ERR_INVALID_ARG, "colour must be 0 or 1");
    if (b_dev == x_dev) return fail(EW_ERR_INVALID_ARG, "b and x may not alias");
    double* tmp = (double*)op->levels[0].x[1];
    if (op->mapped && op->mcoef[0].tw) {
        EW_HIP_TRY(launch_line_half_mapped(x_dev, b_dev, 1.0, op->g, op->mcoef[0], op->a, op->level_relax(0), colour,
                                           op->stream));
        return EW_OK;
    }
    if (op->mapped)
        EW_HIP_TRY(launch_rb_half_mapped(x_dev, tmp, b_dev, 1.0, op->g, op->mcoef[0], op->a, op->level_relax(0), colour,
                                         op->stream));
    else
        EW_HIP_TRY(launch_rb_half<double>(x_dev, tmp, b_dev, 1.0, op->g, op->order, op->a, op->relax, colour, op->stream));
    EW_HIP_TRY(hipMemcpyAsync(x_dev, tmp, op->N * sizeof(double), hipMemcpyDeviceToDevice, op->stream));
    return EW_OK;
}
