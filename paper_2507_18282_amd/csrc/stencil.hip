// Laplacian, explicit leapfrog + filter, implicit update: streaming HIP kernels.
//
// Grid functions hold interior points only (x fastest).  The Dirichlet wall
// value 0 and, for order 4, the odd-reflection ghost u_{-1} = -u_{1} are
// applied while loading neighbours, so no padded copy of the vector (the
// paper's "unpack + apply boundary conditions" step) is ever materialised.
#include "stencil_dev.h"

namespace ew {

// --------------------------------------------------------------------------
// L_h u
// --------------------------------------------------------------------------
template <typename T, int ORDER, int DIM, bool WALLS>
__global__ __launch_bounds__(256) void k_laplacian(const T* __restrict__ u, T* __restrict__ out, Geo g) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, k);
    const T uc = u[c];
    out[c] = lap_at<T, ORDER, DIM, WALLS>(u, c, i, j, k, g, uc);
}

template <typename T>
hipError_t launch_laplacian(const T* u, T* out, const Geo& g, int order, hipStream_t s) {
    dim3 grid = tile_grid(g), block(kTileX, kTileY, 1);
#define EW_LAP(O, D)                                                                   \
    do {                                                                               \
        if (g.wall) k_laplacian<T, O, D, true><<<grid, block, 0, s>>>(u, out, g);      \
        else k_laplacian<T, O, D, false><<<grid, block, 0, s>>>(u, out, g);            \
    } while (0)
    if (g.dim == 2) {
        if (order == 2) EW_LAP(2, 2); else EW_LAP(4, 2);
    } else {
        if (order == 2) EW_LAP(2, 3); else EW_LAP(4, 3);
    }
#undef EW_LAP
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// out = W^{e/2} in with W the Neumann-wall weights (1/2 per Neumann wall the
// point lies on): e = +1 multiplies a wall point by 1/sqrt(2) per wall, e = -1
// by sqrt(2).  W^{1/2} L W^{-1/2} is symmetric, so the eigensolver works on
// vectors y = W^{1/2} u.  in and out may alias.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wall_scale(const double* in, double* out, Geo g, double f) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, k);
    double s = 1.0;
    if (((g.wall & 1) && i == 0) || ((g.wall & 2) && i == g.nx - 1)) s *= f;
    if (((g.wall & 4) && j == 0) || ((g.wall & 8) && j == g.ny - 1)) s *= f;
    if (((g.wall & 16) && k == 0) || ((g.wall & 32) && k == g.nz - 1)) s *= f;
    out[c] = in[c] * s;
}

hipError_t launch_wall_scale(const double* in, double* out, const Geo& g, int e, hipStream_t s) {
    const double f = e > 0 ? 0.70710678118654752440 : 1.41421356237309504880;
    k_wall_scale<<<tile_grid(g), dim3(kTileX, kTileY, 1), 0, s>>>(in, out, g, f);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Explicit leapfrog step fused with the trapezoidal filter accumulation
// (eqs. explicitStep1, explicitScheme, filterQuadrature).  One pass reads
// W^n (stencil), W^{n-1} and the accumulator, and writes W^{n+1} over
// W^{n-1} and the accumulator: 5 values per point.
// --------------------------------------------------------------------------
template <typename T, int ORDER, int DIM, bool FIRST, bool WALLS>
__global__ __launch_bounds__(256) void k_leapfrog(const T* __restrict__ wcur, const T* wprev, T* wnext,
                                                  T* __restrict__ acc, Geo g, T dt2, T ccur, T cnext) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, k);
    const T uc = wcur[c];
    const T lap = lap_at<T, ORDER, DIM, WALLS>(wcur, c, i, j, k, g, uc);
    T wn;
    if (FIRST) {
        wn = uc + (T(0.5) * dt2) * lap;
        acc[c] = ccur * uc + cnext * wn;
    } else {
        wn = T(2) * uc - wprev[c] + dt2 * lap;
        acc[c] = acc[c] + cnext * wn;
    }
    wnext[c] = wn;
}

template <typename T>
hipError_t launch_leapfrog(const T* wcur, const T* wprev, T* wnext, T* acc, const Geo& g, int order, double dt2,
                           double ccur, double cnext, int first, hipStream_t s) {
    dim3 grid = tile_grid(g), block(kTileX, kTileY, 1);
    const T d = (T)dt2, c0 = (T)ccur, c1 = (T)cnext;
#define EW_LF2(O, D, W)                                                                                  \
    do {                                                                                                 \
        if (first) k_leapfrog<T, O, D, true, W><<<grid, block, 0, s>>>(wcur, wprev, wnext, acc, g, d, c0, c1); \
        else k_leapfrog<T, O, D, false, W><<<grid, block, 0, s>>>(wcur, wprev, wnext, acc, g, d, c0, c1);      \
    } while (0)
#define EW_LF(O, D)                   \
    do {                              \
        if (g.wall) EW_LF2(O, D, true); \
        else EW_LF2(O, D, false);       \
    } while (0)
    if (g.dim == 2) {
        if (order == 2) EW_LF(2, 2); else EW_LF(4, 2);
    } else {
        if (order == 2) EW_LF(2, 3); else EW_LF(4, 3);
    }
#undef EW_LF
#undef EW_LF2
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Implicit step update after the solve of M S = 2 W^n (eq. implicitScheme):
// W^{n+1} = S - W^{n-1}, accumulator += c_{n+1} W^{n+1}.  First step
// (eq. implicitStep1): W^1 = S, accumulator = c_0 W^0 + c_1 W^1.
// --------------------------------------------------------------------------
template <typename T, typename TA, bool FIRST>
__global__ __launch_bounds__(256) void k_implicit_update(const T* sol, const T* wprev, T* wnext, TA* __restrict__ acc,
                                                         int64_t n, TA ccur, TA cnext) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        T wn;
        if (FIRST) {
            wn = sol[c];
            acc[c] = ccur * (TA)wprev[c] + cnext * (TA)wn;
        } else {
            wn = sol[c] - wprev[c];
            acc[c] = acc[c] + cnext * (TA)wn;
        }
        wnext[c] = wn;
    }
}

static inline dim3 stream_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

template <typename T, typename TA>
hipError_t launch_implicit_update(const T* sol, const T* wprev, T* wnext, TA* acc, int64_t n, double ccur,
                                  double cnext, int first, hipStream_t s) {
    if (first) k_implicit_update<T, TA, true><<<stream_grid(n), 256, 0, s>>>(sol, wprev, wnext, acc, n, (TA)ccur, (TA)cnext);
    else k_implicit_update<T, TA, false><<<stream_grid(n), 256, 0, s>>>(sol, wprev, wnext, acc, n, (TA)ccur, (TA)cnext);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Elementwise helpers
// --------------------------------------------------------------------------
template <typename TD, typename TS>
__global__ __launch_bounds__(256) void k_convert(TD* __restrict__ dst, const TS* __restrict__ src, int64_t n, TS scale) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        dst[c] = (TD)(scale * src[c]);
}
template <typename TD, typename TS>
hipError_t launch_convert(TD* dst, const TS* src, int64_t n, double scale, hipStream_t s) {
    k_convert<TD, TS><<<stream_grid(n), 256, 0, s>>>(dst, src, n, (TS)scale);
    return hipGetLastError();
}

template <typename T, typename TE>
__global__ __launch_bounds__(256) void k_add_inplace(T* __restrict__ x, const TE* __restrict__ e, int64_t n) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        x[c] = x[c] + (T)e[c];
}
template <typename T, typename TE>
hipError_t launch_add_inplace(T* x, const TE* e, int64_t n, hipStream_t s) {
    k_add_inplace<T, TE><<<stream_grid(n), 256, 0, s>>>(x, e, n);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ x, int64_t n, T v) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        x[c] = v;
}
template <typename T>
hipError_t launch_fill(T* x, int64_t n, T value, hipStream_t s) {
    k_fill<T><<<stream_grid(n), 256, 0, s>>>(x, n, value);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_copy(T* dst, const T* src, int64_t n, double scale, hipStream_t s) {
    k_convert<T, T><<<stream_grid(n), 256, 0, s>>>(dst, src, n, (T)scale);
    return hipGetLastError();
}

#define EW_INST_T(T)                                                                                              \
    template hipError_t launch_laplacian<T>(const T*, T*, const Geo&, int, hipStream_t);                          \
    template hipError_t launch_leapfrog<T>(const T*, const T*, T*, T*, const Geo&, int, double, double, double,   \
                                           int, hipStream_t);                                                     \
    template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                                              \
    template hipError_t launch_scale_copy<T>(T*, const T*, int64_t, double, hipStream_t);
EW_INST_T(double)
EW_INST_T(float)
#undef EW_INST_T
template hipError_t launch_implicit_update<double, double>(const double*, const double*, double*, double*, int64_t,
                                                           double, double, int, hipStream_t);
template hipError_t launch_implicit_update<double, float>(const double*, const double*, double*, float*, int64_t,
                                                          double, double, int, hipStream_t);
template hipError_t launch_convert<float, double>(float*, const double*, int64_t, double, hipStream_t);
template hipError_t launch_convert<double, float>(double*, const float*, int64_t, double, hipStream_t);
template hipError_t launch_convert<double, double>(double*, const double*, int64_t, double, hipStream_t);
template hipError_t launch_add_inplace<double, float>(double*, const float*, int64_t, hipStream_t);
template hipError_t launch_add_inplace<double, double>(double*, const double*, int64_t, hipStream_t);
template hipError_t launch_add_inplace<float, float>(float*, const float*, int64_t, hipStream_t);

}  // namespace ew
