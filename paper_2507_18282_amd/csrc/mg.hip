// Geometric multigrid kernels for the implicit step matrix M = I - a L_h,
// a = dt^2/2 (eq. impMatrix), used with red-black Gauss-Seidel smoothing on
// Cartesian grids.  Levels coarsen by two (n_c = (n-1)/2) and rediscretise the
// same operator; restriction is full weighting and prolongation multilinear.
#include "stencil_dev.h"

namespace ew {

// --------------------------------------------------------------------------
// One red-black half-sweep, out of place: the points whose 0-based index sum
// has parity `colour` get x + (b - M x)/M_ii from the input values, the others
// are copied.  Out of place because for order 4 the +-2 neighbours share the
// colour and must be read before any of them is overwritten.
// --------------------------------------------------------------------------
template <typename T, int ORDER, int DIM, bool WALLS>
__global__ __launch_bounds__(256) void k_rb_half(const T* __restrict__ xin, T* __restrict__ xout,
                                                 const T* __restrict__ b, T bscale, Geo g, T a, T w,
                                                 int colour) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, k);
    const T xc = xin[c];
    if (((i + j + k) & 1) != colour) {
        xout[c] = xc;
        return;
    }
    const T lap = lap_at<T, ORDER, DIM, WALLS>(xin, c, i, j, k, g, xc);
    const T r = bscale * b[c] - (xc - a * lap);
    xout[c] = xc + (w * r) / mdiag_at<T, ORDER, DIM, WALLS>(i, j, k, g, a);
}

template <typename T>
hipError_t launch_rb_half(const T* xin, T* xout, const T* b, double bscale, const Geo& g, int order, double a,
                          double w, int colour, hipStream_t s) {
    dim3 grid = tile_grid(g), block(kTileX, kTileY, 1);
    const T bs = (T)bscale, aa = (T)a, ww = (T)w;
#define EW_RB(O, D)                                                                                   \
    do {                                                                                              \
        if (g.wall) k_rb_half<T, O, D, true><<<grid, block, 0, s>>>(xin, xout, b, bs, g, aa, ww, colour);  \
        else k_rb_half<T, O, D, false><<<grid, block, 0, s>>>(xin, xout, b, bs, g, aa, ww, colour);       \
    } while (0)
    if (g.dim == 2) {
        if (order == 2) EW_RB(2, 2); else EW_RB(4, 2);
    } else {
        if (order == 2) EW_RB(2, 3); else EW_RB(4, 3);
    }
#undef EW_RB
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Prolongation (multilinear) fused with the correction x += P xc.  Along an
// axis whose low wall is Dirichlet the coarse point I sits at fine index
// 2I + 1; behind a Neumann low wall (an active wall point) at 2I.  Fine points
// between coarse points take the mean of their two neighbours; a neighbour
// beyond a Dirichlet wall is the wall value 0 (a Neumann wall point is itself
// a coarse point, so no neighbour lies beyond it).
// --------------------------------------------------------------------------
__device__ __forceinline__ void interp_1d(int f, int nc, int off, int& c0, int& c1, float& w0, float& w1) {
    const int q = f - off;
    if (q >= 0 && !(q & 1)) {  // coincides with coarse point q/2
        c0 = q >> 1;
        c1 = -1;
        w0 = 1.0f;
        w1 = 0.0f;
    } else {                   // midway between coarse (q-1)/2 and (q+1)/2
        c0 = (q - 1) >> 1;
        c1 = c0 + 1;
        w0 = 0.5f;
        w1 = 0.5f;
        if (c1 >= nc) c1 = -1;
    }
}

// Without branches: an absent neighbour (beyond a wall or the last coarse
// point) is read at a valid index with weight 0, so every lane issues the
// same loads (skipping it would branch on the parity of i, j and k within a
// wavefront; on the 2047^2 mapped level that form took 29.8 us, this one
// 22.3).  Adding a zero-weighted term leaves the sum unchanged.
__device__ __forceinline__ void interp_1d_safe(int f, int nc, int off, int& c0, int& c1, float& w0, float& w1) {
    interp_1d(f, nc, off, c0, c1, w0, w1);
    if (c0 < 0) { c0 = 0; w0 = 0.0f; }
    if (c1 < 0) { c1 = 0; w1 = 0.0f; }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_correct_nb(T* __restrict__ x, const T* __restrict__ xc, Geo gf,
                                                            Geo gc) {
    int i, j, k;
    if (!tile_coords(gf, i, j, k)) return;
    int xi0, xi1, yj0, yj1, zk0 = 0, zk1 = 0;
    float wx0, wx1, wy0, wy1, wz0 = 1.0f, wz1 = 0.0f;
    interp_1d_safe(i, gc.nx, (gf.wall & 1) ? 0 : 1, xi0, xi1, wx0, wx1);
    interp_1d_safe(j, gc.ny, (gf.wall & 4) ? 0 : 1, yj0, yj1, wy0, wy1);
    if (DIM == 3) interp_1d_safe(k, gc.nz, (gf.wall & 16) ? 0 : 1, zk0, zk1, wz0, wz1);
    auto plane = [&](int kc) -> T {
        const T* r0 = xc + ((int64_t)kc * gc.ny + yj0) * gc.nx;
        const T* r1 = xc + ((int64_t)kc * gc.ny + yj1) * gc.nx;
        const T row0 = (T)wx0 * r0[xi0] + (T)wx1 * r0[xi1];
        const T row1 = (T)wx0 * r1[xi0] + (T)wx1 * r1[xi1];
        return (T)wy0 * row0 + (T)wy1 * row1;
    };
    T v = plane(zk0);
    if (DIM == 3) v = (T)wz0 * v + (T)wz1 * plane(zk1);
    const int64_t cf = lin(gf, i, j, k);
    x[cf] = x[cf] + v;
}

template <typename T>
hipError_t launch_prolong_correct(T* x, const T* xc, const Geo& gf, const Geo& gc, hipStream_t s) {
    dim3 grid = tile_grid(gf), block(kTileX, kTileY, 1);
    if (gf.dim == 2) k_prolong_correct_nb<T, 2><<<grid, block, 0, s>>>(x, xc, gf, gc);
    else k_prolong_correct_nb<T, 3><<<grid, block, 0, s>>>(x, xc, gf, gc);
    return hipGetLastError();
}

#define EW_INST_MG(T)                                                                                          \
    template hipError_t launch_rb_half<T>(const T*, T*, const T*, double, const Geo&, int, double, double, int, \
                                          hipStream_t);                                                        \
    template hipError_t launch_prolong_correct<T>(T*, const T*, const Geo&, const Geo&, hipStream_t);
EW_INST_MG(double)
EW_INST_MG(float)
#undef EW_INST_MG

}  // namespace ew
