// A single curvilinear grid by the mapping method (Sec. "Discrete
// approximations"): the order-2 Laplacian in conservative form,
//
//   J L_h u = D+r (A11 D-r u) + D+s (A22 D-s u) + D0r (B D0s u) + D0s (B D0r u),
//
// J = x_r y_s - x_s y_r, J a^11 = (x_s^2 + y_s^2)/J, J a^22 = (x_r^2 + y_r^2)/J,
// B = J a^12 = -(x_r x_s + y_r y_s)/J, A11 (A22) at a half point the mean of
// J a^11 (J a^22) at its two nodes, metric derivatives by centred differences
// of the grid coordinates, Dirichlet walls (u = 0).  J L_h is symmetric, so
// L_h is self-adjoint in the inner product weighted by J; the eigensolver
// works in y = J^{1/2} u.
//
// The coefficients are built once on the host from the caller's coordinates
// and kept on the device as four arrays (A11 / dr^2 at x half points, A22 /
// ds^2 at y half points, B / (4 dr ds) and 1/J at the nodes): the leapfrog
// step streams them with the three state arrays, 72 B per point-step.
#include <cmath>
#include <memory>
#include <vector>

#include "op.h"
#include "stencil_dev.h"

namespace ew {

// L_h u at active point (i, j), c = j nx + i; values beyond the walls are 0.
// A cross term whose node lies on a wall multiplies a difference of wall
// values, so it is dropped rather than read.
__device__ __forceinline__ double lap_mapped(const double* __restrict__ u, int64_t c, int i, int j, const Geo& g,
                                             const MapCoef& m) {
    const int nx = g.nx;
    const bool w = i > 0, e = i < nx - 1, s = j > 0, n = j < g.ny - 1;
    const double uc = u[c];
    const double uW = w ? u[c - 1] : 0.0, uE = e ? u[c + 1] : 0.0;
    const double uS = s ? u[c - nx] : 0.0, uN = n ? u[c + nx] : 0.0;
    const double uSW = (w && s) ? u[c - nx - 1] : 0.0, uSE = (e && s) ? u[c - nx + 1] : 0.0;
    const double uNW = (w && n) ? u[c + nx - 1] : 0.0, uNE = (e && n) ? u[c + nx + 1] : 0.0;
    const int64_t hw = (int64_t)j * (nx + 1) + i;  // half point i - 1/2
    double t = m.cw[hw + 1] * (uE - uc) - m.cw[hw] * (uc - uW);
    t += m.cs[c + nx] * (uN - uc) - m.cs[c] * (uc - uS);
    const double bE = e ? m.cb[c + 1] : 0.0, bW = w ? m.cb[c - 1] : 0.0;
    const double bN = n ? m.cb[c + nx] : 0.0, bS = s ? m.cb[c - nx] : 0.0;
    t += bE * (uNE - uSE) - bW * (uNW - uSW);  // D0r (B D0s u)
    t += bN * (uNE - uNW) - bS * (uSE - uSW);  // D0s (B D0r u)
    return m.ij[c] * t;
}

__global__ __launch_bounds__(256) void k_laplacian_mapped(const double* __restrict__ u, double* __restrict__ out,
                                                          Geo g, MapCoef m) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, 0);
    out[c] = lap_mapped(u, c, i, j, g, m);
}

// Leapfrog step fused with the filter accumulation (eqs. explicitStep1,
// explicitScheme, filterQuadrature), as k_leapfrog.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_leapfrog_mapped(const double* __restrict__ wcur, const double* wprev,
                                                         double* wnext, double* __restrict__ acc, Geo g, MapCoef m,
                                                         double dt2, double ccur, double cnext) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, 0);
    const double uc = wcur[c];
    const double lap = lap_mapped(wcur, c, i, j, g, m);
    double wn;
    if (FIRST) {
        wn = uc + (0.5 * dt2) * lap;
        acc[c] = ccur * uc + cnext * wn;
    } else {
        wn = 2.0 * uc - wprev[c] + dt2 * lap;
        acc[c] = acc[c] + cnext * wn;
    }
    wnext[c] = wn;
}

__global__ __launch_bounds__(256) void k_pointwise_mul(const double* in, const double* __restrict__ f, double* out,
                                                       int64_t n) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        out[c] = in[c] * f[c];
}

hipError_t launch_laplacian_mapped(const double* u, double* out, const Geo& g, const MapCoef& m, hipStream_t s) {
    k_laplacian_mapped<<<tile_grid(g), dim3(kTileX, kTileY, 1), 0, s>>>(u, out, g, m);
    return hipGetLastError();
}

hipError_t launch_leapfrog_mapped(const double* wcur, const double* wprev, double* wnext, double* acc, const Geo& g,
                                  const MapCoef& m, double dt2, double ccur, double cnext, int first, hipStream_t s) {
    const dim3 grid = tile_grid(g), block(kTileX, kTileY, 1);
    if (first) k_leapfrog_mapped<true><<<grid, block, 0, s>>>(wcur, wprev, wnext, acc, g, m, dt2, ccur, cnext);
    else k_leapfrog_mapped<false><<<grid, block, 0, s>>>(wcur, wprev, wnext, acc, g, m, dt2, ccur, cnext);
    return hipGetLastError();
}

hipError_t launch_pointwise_mul(const double* in, const double* f, double* out, int64_t n, hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    k_pointwise_mul<<<(unsigned)b, 256, 0, s>>>(in, f, out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host: coefficients from the coordinates.  xy holds x then y, each
// (n1 + 4) x (n2 + 4) with node (i, j), i in [-2, n1 + 1], at (i + 2) +
// (n1 + 4)(j + 2); metric terms are formed at the nodes i in [-1, n1],
// j in [-1, n2] (walls included).
// ---------------------------------------------------------------------------
namespace {

struct HostCoef {
    std::vector<double> cw, cs, cb, ij, sq, isq;
    double rho = 0.0;
};

ew_status build_coefficients(const double* xy, int n1, int n2, HostCoef& hc) {
    const int64_t px = n1 + 4, plane = px * (int64_t)(n2 + 4);
    for (int64_t q = 0; q < 2 * plane; ++q)
        if (!std::isfinite(xy[q])) return fail(EW_ERR_INVALID_ARG, "mapped grid coordinates must be finite");
    const double dr = 1.0 / (n1 + 1), ds = 1.0 / (n2 + 1);
    auto X = [&](int i, int j) { return xy[(i + 2) + px * (j + 2)]; };
    auto Y = [&](int i, int j) { return xy[plane + (i + 2) + px * (j + 2)]; };
    // node arrays over i in [-1, n1], j in [-1, n2]: index (i + 1) + (n1 + 2)(j + 1)
    const int64_t nx2 = n1 + 2, ny2 = n2 + 2;
    std::vector<double> J(nx2 * ny2), a11(nx2 * ny2), a22(nx2 * ny2), a12(nx2 * ny2);
    for (int j = -1; j <= n2; ++j)
        for (int i = -1; i <= n1; ++i) {
            const double xr = (X(i + 1, j) - X(i - 1, j)) / (2.0 * dr), yr = (Y(i + 1, j) - Y(i - 1, j)) / (2.0 * dr);
            const double xs = (X(i, j + 1) - X(i, j - 1)) / (2.0 * ds), ys = (Y(i, j + 1) - Y(i, j - 1)) / (2.0 * ds);
            const double jac = xr * ys - xs * yr;
            if (!(jac > 0.0) || !std::isfinite(jac))
                return fail(EW_ERR_INVALID_ARG, "mapped grid: the Jacobian x_r y_s - x_s y_r must be positive at every "
                                                "node (walls included)");
            const int64_t q = (i + 1) + nx2 * (j + 1);
            J[q] = jac;
            a11[q] = (xs * xs + ys * ys) / jac;
            a22[q] = (xr * xr + yr * yr) / jac;
            a12[q] = -(xr * xs + yr * ys) / jac;
        }
    auto node = [&](const std::vector<double>& F, int i, int j) { return F[(i + 1) + nx2 * (j + 1)]; };
    const int64_t N = (int64_t)n1 * n2;
    hc.cw.assign((int64_t)(n1 + 1) * n2, 0.0);
    hc.cs.assign((int64_t)n1 * (n2 + 1), 0.0);
    hc.cb.assign(N, 0.0);
    hc.ij.assign(N, 0.0);
    hc.sq.assign(N, 0.0);
    hc.isq.assign(N, 0.0);
    const double idr2 = 1.0 / (dr * dr), ids2 = 1.0 / (ds * ds), q4 = 1.0 / (4.0 * dr * ds);
    for (int j = 0; j < n2; ++j)
        for (int hi = 0; hi <= n1; ++hi)
            hc.cw[hi + (int64_t)(n1 + 1) * j] = 0.5 * (node(a11, hi - 1, j) + node(a11, hi, j)) * idr2;
    for (int hj = 0; hj <= n2; ++hj)
        for (int i = 0; i < n1; ++i)
            hc.cs[i + (int64_t)n1 * hj] = 0.5 * (node(a22, i, hj - 1) + node(a22, i, hj)) * ids2;
    double rho = 0.0;
    for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n1; ++i) {
            const int64_t c = i + (int64_t)n1 * j;
            const double jac = node(J, i, j);
            hc.cb[c] = node(a12, i, j) * q4;
            hc.ij[c] = 1.0 / jac;
            hc.sq[c] = std::sqrt(jac);
            hc.isq[c] = 1.0 / hc.sq[c];
            // Gershgorin: (1/J) times the absolute sum of the nine weights of
            // J L_h, the cross weights of wall nodes included
            const double wE = hc.cw[(i + 1) + (int64_t)(n1 + 1) * j], wW = hc.cw[i + (int64_t)(n1 + 1) * j];
            const double wN = hc.cs[i + (int64_t)n1 * (j + 1)], wS = hc.cs[c];
            const double bE = node(a12, i + 1, j) * q4, bW = node(a12, i - 1, j) * q4;
            const double bN = node(a12, i, j + 1) * q4, bS = node(a12, i, j - 1) * q4;
            const double sum = std::fabs(wE + wW + wN + wS) + std::fabs(wE) + std::fabs(wW) + std::fabs(wN) +
                               std::fabs(wS) + std::fabs(bE + bN) + std::fabs(bE + bS) + std::fabs(bW + bN) +
                               std::fabs(bW + bS);
            rho = std::max(rho, sum / jac);
        }
    hc.rho = rho;
    return EW_OK;
}

ew_status upload(Op* op, const std::vector<double>& h, const double** dst) {
    double* d = nullptr;
    EW_TRY(op->alloc((void**)&d, h.size() * sizeof(double)));
    EW_HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    *dst = d;
    return EW_OK;
}

}  // namespace
}  // namespace ew

using namespace ew;

extern "C" ew_status ew_op_create_mapped(const ew_grid_desc* grid, const ew_op_desc* desc, const double* xy_host,
                                         void* hip_stream, ew_op* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!xy_host) return fail(EW_ERR_INVALID_ARG, "mapped grid coordinates are null");
    EW_TRY(validate_descs(grid, desc));
    if (grid->dim != 2) return fail(EW_ERR_UNSUPPORTED, "mapped grids are two-dimensional");
    if (grid->order != 2) return fail(EW_ERR_UNSUPPORTED, "mapped grids use the order-2 operator");
    for (int e = 0; e < 2; ++e)
        if (grid->walls[0][e] != EW_WALL_DIRICHLET || grid->walls[1][e] != EW_WALL_DIRICHLET)
            return fail(EW_ERR_UNSUPPORTED, "mapped grids have Dirichlet walls");
    if (desc->ts != EW_TS_EXPLICIT) return fail(EW_ERR_UNSUPPORTED, "mapped grids use explicit time-stepping");
    if (desc->precision != EW_PREC_FP64) return fail(EW_ERR_UNSUPPORTED, "mapped grids run in FP64");
    const int n1 = (int)grid->n[0], n2 = (int)grid->n[1];
    HostCoef hc;
    EW_TRY(build_coefficients(xy_host, n1, n2, hc));

    std::unique_ptr<ew_op_s> op(new ew_op_s());
    op->dim = 2;
    op->order = 2;
    op->n[0] = n1;
    op->n[1] = n2;
    op->n[2] = 1;
    op->h[0] = 1.0 / (n1 + 1);  // parameter-space spacings
    op->h[1] = 1.0 / (n2 + 1);
    op->desc = *desc;
    op->stream = (hipStream_t)hip_stream;
    op->g = make_geo(2, op->n, op->h, 0);
    op->N = op->g.size();
    EW_HIP_TRY(hipGetDevice(&op->device));
    op->mapped = true;
    op->map_rho = hc.rho;
    TimePlan tp;
    make_time_plan(2, 2, op->h, op->desc, tp, hc.rho);
    op->omega_used = tp.omega_used;
    op->t_final = tp.t_final;
    op->n_t = tp.n_t;
    op->dt = tp.dt;
    op->alpha_d = tp.alpha_d;
    op->c = tp.c;
    op->a = 0.5 * op->dt * op->dt;
    EW_TRY(upload(op.get(), hc.cw, &op->mc.cw));
    EW_TRY(upload(op.get(), hc.cs, &op->mc.cs));
    EW_TRY(upload(op.get(), hc.cb, &op->mc.cb));
    EW_TRY(upload(op.get(), hc.ij, &op->mc.ij));
    EW_TRY(upload(op.get(), hc.sq, &op->mc.sq));
    EW_TRY(upload(op.get(), hc.isq, &op->mc.isq));
    const int64_t N = op->N;
    EW_TRY(op->alloc((void**)&op->partial_dev, kRedBlocks * sizeof(double) * 4));
    EW_HIP_TRY(hipHostMalloc((void**)&op->partial_host, kRedBlocks * sizeof(double) * 4, hipHostMallocDefault));
    EW_TRY(op->alloc((void**)&op->wA, N * sizeof(double)));
    EW_TRY(op->alloc((void**)&op->wB, N * sizeof(double)));
    EW_TRY(op->alloc((void**)&op->c_dev, op->c.size() * sizeof(double)));
    EW_HIP_TRY(hipMemcpy(op->c_dev, op->c.data(), op->c.size() * sizeof(double), hipMemcpyHostToDevice));
    *out = op.release();
    return EW_OK;
}

extern "C" ew_status ew_op_mapped_rho(ew_op op, double* rho_host) {
    if (!op || !rho_host) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (!op->mapped) return fail(EW_ERR_INVALID_ARG, "operator is not on a mapped grid");
    *rho_host = op->map_rho;
    return EW_OK;
}
