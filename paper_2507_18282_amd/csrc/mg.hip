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

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong_correct(T* __restrict__ x, const T* __restrict__ xc, Geo gf, Geo gc) {
    int i, j, k;
    if (!tile_coords(gf, i, j, k)) return;
    int xi[2], yj[2], zk[2];
    float wx[2], wy[2], wz[2];
    // offsets 1 behind a Dirichlet low wall, 0 behind a Neumann one
    interp_1d(i, gc.nx, (gf.wall & 1) ? 0 : 1, xi[0], xi[1], wx[0], wx[1]);
    interp_1d(j, gc.ny, (gf.wall & 4) ? 0 : 1, yj[0], yj[1], wy[0], wy[1]);
    if (DIM == 3) interp_1d(k, gc.nz, (gf.wall & 16) ? 0 : 1, zk[0], zk[1], wz[0], wz[1]);
    else { zk[0] = 0; zk[1] = -1; wz[0] = 1.0f; wz[1] = 0.0f; }
    T v = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (zk[c] < 0) continue;
        T plane = T(0);
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            if (yj[bb] < 0) continue;
            T row = T(0);
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
                if (xi[aa] < 0) continue;
                row += (T)wx[aa] * xc[lin(gc, xi[aa], yj[bb], zk[c])];
            }
            plane += (T)wy[bb] * row;
        }
        v += (T)wz[c] * plane;
    }
    const int64_t cf = lin(gf, i, j, k);
    x[cf] = x[cf] + v;
}

template <typename T>
hipError_t launch_prolong_correct(T* x, const T* xc, const Geo& gf, const Geo& gc, hipStream_t s) {
    dim3 grid = tile_grid(gf), block(kTileX, kTileY, 1);
    if (gf.dim == 2) k_prolong_correct<T, 2><<<grid, block, 0, s>>>(x, xc, gf, gc);
    else k_prolong_correct<T, 3><<<grid, block, 0, s>>>(x, xc, gf, gc);
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
