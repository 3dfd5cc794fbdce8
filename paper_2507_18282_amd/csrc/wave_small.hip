// Explicit wave-solve of a small 2D grid in one workgroup: the leapfrog
// scheme (eq. explicitScheme, first step eq. explicitStep1) with the
// trapezoidal filter accumulated in the same loop (eq. filterQuadrature).
// W^n lives in LDS with a zero frame of two cells (the Dirichlet wall and the
// cells the order-4 stencil reaches beyond it), double-buffered so that a step
// needs one barrier; W^{n-1}, the accumulator and the point coordinates stay
// in registers.  With STRIP (order 2, Dirichlet walls, nx dividing the
// thread count) a thread owns PTS consecutive points of one column, so the
// vertical neighbours inside its strip come from registers and a step reads
// LDS 10 instead of 16 times per thread: one workgroup is LDS-bandwidth
// bound.  All N_t steps run in one launch,
// so the grid never goes back to HBM between reading v and writing S v: on
// grids of a few thousand points the per-step launches of the tiled leapfrog
// are pure latency.
#include "op.h"
#include "stencil_dev.h"

namespace ew {
namespace {

constexpr int kSmallThreads = 1024;

template <typename T, int ORDER, int PTS, bool STRIP>
__global__ __launch_bounds__(kSmallThreads) void k_wave_small(const double* __restrict__ v, double* __restrict__ out,
                                                              Geo g, T dt2, const double* __restrict__ c, int n_t) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, ny = g.ny, px = nx + 4, n = nx * ny, nl = px * (ny + 4);
    T* Xs = reinterpret_cast<T*>(smem);  // W^n
    T* Xn = Xs + nl;                      // W^{n+1}
    const int tid = threadIdx.x;
    const T cx = ORDER == 2 ? (T)g.ihx2 : (T)(g.ihx2 / 12.0);
    const T cy = ORDER == 2 ? (T)g.ihy2 : (T)(g.ihy2 / 12.0);
    for (int q = tid; q < 2 * nl; q += kSmallThreads) Xs[q] = T(0);
    __syncthreads();
    T cur[PTS], prev[PTS], acc[PTS];
    int lp[PTS], lij[PTS];  // LDS index; i | j << 16
    const T c0 = (T)c[0];
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        int q, i, j;
        if (STRIP) {
            i = tid % nx;
            j = (tid / nx) * PTS + t;
            q = j < ny ? j * nx + i : n;
        } else {
            q = tid + t * kSmallThreads;
            i = q % nx;
            j = q / nx;
        }
        lp[t] = -1;
        cur[t] = T(0);  // a point beyond the grid reads as the wall's 0
        prev[t] = T(0);
        acc[t] = T(0);
        if (q < n) {
            lij[t] = i | (j << 16);
            lp[t] = (j + 2) * px + i + 2;
            cur[t] = (T)v[q];
            prev[t] = cur[t];
            acc[t] = c0 * cur[t];
            Xs[lp[t]] = cur[t];
        }
    }
    __syncthreads();
    for (int step = 0; step < n_t; ++step) {
        const T cn = (T)c[step + 1];
        T nxt[PTS];
#pragma unroll
        for (int t = 0; t < PTS; ++t) {
            nxt[t] = cur[t];
            if (lp[t] < 0) continue;
            const int p = lp[t];
            const T uc = cur[t];
            T lap;
            if (STRIP) {
                const T dn = t > 0 ? cur[t - 1] : Xs[p - px];
                const T up = t < PTS - 1 ? cur[t + 1] : Xs[p + px];
                lap = (Xs[p - 1] + Xs[p + 1] - T(2) * uc) * cx + (dn + up - T(2) * uc) * cy;
            } else if (ORDER == 2 && g.wall == 0) {
                lap = (Xs[p - 1] + Xs[p + 1] - T(2) * uc) * cx + (Xs[p - px] + Xs[p + px] - T(2) * uc) * cy;
            } else {
                // wall closures (Dirichlet odd reflection, Neumann even
                // reflection) replace the frame's zeros
                const int i = lij[t] & 0xFFFF, j = lij[t] >> 16;
                lap = d2_framed<T, ORDER>(Xs, p, 1, i, nx, uc, g.wall & 3) * cx +
                      d2_framed<T, ORDER>(Xs, p, px, j, ny, uc, (g.wall >> 2) & 3) * cy;
            }
            const T nw = (step == 0) ? uc + (T(0.5) * dt2) * lap : T(2) * uc - prev[t] + dt2 * lap;
            acc[t] += cn * nw;
            Xn[p] = nw;
            prev[t] = uc;
            nxt[t] = nw;
        }
#pragma unroll
        for (int t = 0; t < PTS; ++t) cur[t] = nxt[t];  // the strip's neighbours were read old
        __syncthreads();  // W^{n+1} complete; W^n no longer read
        T* sw = Xs;
        Xs = Xn;
        Xn = sw;
    }
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        if (lp[t] < 0) continue;
        const int i = lij[t] & 0xFFFF, j = lij[t] >> 16;
        out[j * nx + i] = (double)acc[t];
    }
}

template <typename T>
constexpr int small_pts_max() {
    return 8;  // keeps the per-thread state within the 1024-thread register budget (no spills)
}

template <typename T, int ORDER, int PTS, bool STRIP>
hipError_t launch_small_as(const double* v, double* out, const Geo& g, double dt2, const double* c, int n_t,
                           hipStream_t s) {
    const size_t lds = 2 * (size_t)(g.nx + 4) * (g.ny + 4) * sizeof(T);
    const void* f = (const void*)k_wave_small<T, ORDER, PTS, STRIP>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_wave_small<T, ORDER, PTS, STRIP><<<1, kSmallThreads, lds, s>>>(v, out, g, (T)dt2, c, n_t);
    return hipGetLastError();
}

// Strips of PTS rows per column when nx divides the thread count and the
// strips cover every row (order 2, Dirichlet walls).
template <typename T, int ORDER, int PTS>
hipError_t launch_small(const double* v, double* out, const Geo& g, double dt2, const double* c, int n_t,
                        hipStream_t s) {
    if (ORDER == 2 && g.wall == 0 && kSmallThreads % g.nx == 0 && (int64_t)(kSmallThreads / g.nx) * PTS >= g.ny)
        return launch_small_as<T, ORDER, PTS, ORDER == 2>(v, out, g, dt2, c, n_t, s);
    return launch_small_as<T, ORDER, PTS, false>(v, out, g, dt2, c, n_t, s);
}

}  // namespace

template <typename T>
bool wave_small_fits(const Geo& g) {
    const int64_t n = g.size();
    return g.dim == 2 && n <= (int64_t)small_pts_max<T>() * kSmallThreads &&
           2 * (int64_t)(g.nx + 4) * (g.ny + 4) * (int64_t)sizeof(T) <= (int64_t)kCoarseMaxLdsBytes;
}

template <typename T>
hipError_t launch_wave_small(const double* v, double* out, const Geo& g, int order, double dt2, const double* c_dev,
                             int n_t, hipStream_t s) {
    if (!wave_small_fits<T>(g)) return hipErrorInvalidValue;
    const int64_t n = g.size();
    constexpr int PM = small_pts_max<T>();
    if (order == 2) {
        if (n <= 4 * kSmallThreads) return launch_small<T, 2, 4>(v, out, g, dt2, c_dev, n_t, s);
        return launch_small<T, 2, PM>(v, out, g, dt2, c_dev, n_t, s);
    }
    if (n <= 4 * kSmallThreads) return launch_small<T, 4, 4>(v, out, g, dt2, c_dev, n_t, s);
    return launch_small<T, 4, PM>(v, out, g, dt2, c_dev, n_t, s);
}

template bool wave_small_fits<double>(const Geo&);
template bool wave_small_fits<float>(const Geo&);
template hipError_t launch_wave_small<double>(const double*, double*, const Geo&, int, double, const double*, int,
                                              hipStream_t);
template hipError_t launch_wave_small<float>(const double*, double*, const Geo&, int, double, const double*, int,
                                             hipStream_t);

}  // namespace ew
