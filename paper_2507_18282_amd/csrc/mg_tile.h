// Declarations of the LDS-tiled multigrid kernels (mg_tile.hip).
#pragma once

#include "ew_internal.h"

namespace ew {

// Levels handled by the single-workgroup coarse kernel.  Level arrays live in
// dynamic LDS at the given element offsets, each padded by two zero cells per
// side.  The first such level must have nx, ny <= 64 in 2D, or nx, ny, nz <= 16
// in 3D (the kernel's fixed thread-to-column map).
constexpr int kMaxCoarseLevels = 16;
constexpr int kCoarseMax2D = 64;
constexpr int kCoarseMax3D = 16;
constexpr size_t kCoarseMaxLdsBytes = 160 * 1024;
struct CoarseLevels {
    int nlev;
    int lds_elems;
    int off_r;  // scratch residual array, sized for level 0
    int off_x[kMaxCoarseLevels];
    int off_b[kMaxCoarseLevels];
    Geo g[kMaxCoarseLevels];
};

// True where the 3D sweep of level g (stencil order `order`) marches through
// z and applies the prolongation inside the sweep (launch_sweep_tile with
// prolong); elsewhere 3D V-cycles prolong in a pass of their own.
bool sweep_z3d_fuses_prolong(const Geo& g, int order);

// One full red-black sweep xout = RB(xin (+ P xc if prolong), bscale b), tile by tile;
// every relaxed point gets x + w (b - M x)_i / M_ii (w: relaxation weight).
// xin is not read when zero_in.  xin and xout must not alias.
// ev0/ev1 (may be null) are recorded at the start and end of the sweep's dispatch.
template <typename T>
hipError_t launch_sweep_tile(const T* xin, const T* xc, const T* b, double bscale, T* xout, const Geo& g,
                             const Geo& gc, int order, double a, double w, bool zero_in, bool prolong,
                             hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// bc = full-weighting restriction of the residual bscale b - M x.
template <typename T>
hipError_t launch_restrict_tile(const T* x, const T* b, double bscale, const Geo& gf, int order, double a, T* bc,
                                const Geo& gc, hipStream_t s);
// V-cycle over the levels of c in one workgroup; x_in may be null (zero start).
// w0: relaxation weight of c's first level, w: of the others (a level of one
// point uses 1).
template <typename T>
hipError_t launch_coarse_vcycle(const T* b, double bscale, const T* x_in, T* x_out, const CoarseLevels& c, int order,
                                double a, double w0, double w, int nu1, int nu2, int coarse_sweeps, hipStream_t s);
template <typename T>
hipError_t prepare_coarse_vcycle(int dim, int order, size_t lds_bytes);
// Residual norm by tiles: tile_partial (residual_tiles(g) doubles) receives
// the sum of r^2, r = bscale b - M x, per tile, and partial (kRedBlocks
// doubles) the tile sums folded in a fixed order; with r_out != nullptr the
// residual is stored too, converted to TR.
int64_t residual_tiles(const Geo& g);
template <typename T, typename TR>
hipError_t launch_residual_tile(const T* x, const T* b, double bscale, const Geo& g, int order, double a,
                                double* tile_partial, double* partial, TR* r_out, hipStream_t s);
// 2D grids (sweep2d.hip).  launch_sweep2x2d: two consecutive red-black
// sweeps of a 2D level in one pass, out of place (xin may be null with zero_in).
template <typename T>
hipError_t launch_sweep2x2d(const T* xin, const T* b, double bscale, T* xout, const Geo& g, int order, double a,
                            double w, bool zero_in, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// launch_sweep2x_restrict2d: the same two sweeps, then from the same staging
// bc = full-weighting restriction of the residual bscale b - M xout (what
// launch_restrict_tile computes from xout); 2D levels without Neumann walls
// whose coarse level gc has (n-1)/2 points per direction.
template <typename T>
hipError_t launch_sweep2x_restrict2d(const T* xin, const T* b, double bscale, T* xout, const Geo& g, int order,
                                     double a, double w, bool zero_in, T* bc, const Geo& gc, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
hipError_t launch_sweep2d(const T* xin, const T* xc, const T* b, double bscale, T* xout, const Geo& g, const Geo& gc,
                          int order, double a, double w, bool zero_in, bool prolong, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1);

}  // namespace ew
