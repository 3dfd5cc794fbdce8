// Device helpers: thread-to-point mapping, stencils with the wall closure,
// the diagonal of M = I - a L, and deterministic block reductions.
#pragma once

#include "ew_internal.h"

namespace ew {

constexpr int kTileX = 64;  // one wavefront along x: coalesced rows
constexpr int kTileY = 4;

__host__ inline dim3 tile_grid(const Geo& g) {
    return dim3((unsigned)((g.nx + kTileX - 1) / kTileX), (unsigned)((g.ny + kTileY - 1) / kTileY), (unsigned)g.nz);
}

// Block coordinates of a launch renumbered so that each XCD (workgroup w
// runs on XCD w % 8) takes one contiguous band of tile rows (of tile planes
// in 3D): the rows a tile shares with its neighbours are then fetched into
// that XCD's L2 once.
__device__ __forceinline__ void xcd_block(int& bx, int& by, int& bz) {
    constexpr int kXcds = 8;
    const int gx = gridDim.x, gy = gridDim.y, nb = gridDim.x * gridDim.y * gridDim.z;
    const int w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int x = w % kXcds, q = nb / kXcds, r = nb % kXcds;
    const int t = x * q + (x < r ? x : r) + w / kXcds;  // a bijection of [0, nb)
    bx = t % gx;
    by = (t / gx) % gy;
    bz = t / (gx * gy);
}

__device__ __forceinline__ void xcd_block(int& bx, int& by) {
    int bz;
    xcd_block(bx, by, bz);
}

// Point (i, j, k) of a thread in a launch of tile_grid, tiles in XCD order.
__device__ __forceinline__ bool tile_coords(const Geo& g, int& i, int& j, int& k) {
    int bx, by;
    xcd_block(bx, by, k);
    i = bx * kTileX + threadIdx.x;
    j = by * kTileY + threadIdx.y;
    return i < g.nx && j < g.ny;
}

__device__ __forceinline__ int64_t lin(const Geo& g, int i, int j, int k) {
    return ((int64_t)k * g.ny + j) * g.nx + i;
}

// Second difference along one axis at index i (0-based) of n active points,
// un-scaled: order 2 returns u_{i-1} - 2u_i + u_{i+1}; order 4 returns
// -u_{i-2} + 16u_{i-1} - 30u_i + 16u_{i+1} - u_{i+2}.  w holds the axis's
// Neumann walls (bit 0 low, bit 1 high).  Beyond a Dirichlet wall index -1
// (or n) is the wall, value 0, and index -2 (or n+1) the odd-reflection ghost
// -u_0 (or -u_{n-1}); beyond a Neumann wall ghosts mirror evenly about the
// wall point, u_{-k} = u_k (u_{n-1+k} = u_{n-1-k}).
template <typename T, int ORDER>
__device__ __forceinline__ T d2_axis(const T* __restrict__ u, int64_t c, int i, int n, int64_t stride, T uc,
                                     int w = 0) {
    const bool nlo = (w & 1) != 0, nhi = (w & 2) != 0;
    const T l1 = (i > 0) ? u[c - stride] : (nlo ? u[c + stride] : T(0));
    const T r1 = (i < n - 1) ? u[c + stride] : (nhi ? u[c - stride] : T(0));
    if (ORDER == 2) {
        return l1 + r1 - T(2) * uc;
    } else {
        T l2, r2;
        if (i > 1) l2 = u[c - 2 * stride];
        else if (i == 1) l2 = nlo ? uc : T(0);
        else l2 = nlo ? u[c + 2 * stride] : -uc;
        if (i < n - 2) r2 = u[c + 2 * stride];
        else if (i == n - 2) r2 = nhi ? uc : T(0);
        else r2 = nhi ? u[c - 2 * stride] : -uc;
        return T(16) * (l1 + r1) - (l2 + r2) - T(30) * uc;
    }
}

// The same from a buffer whose neighbours beyond the walls read as 0 (an LDS
// frame): the wall closures replace those values.
template <typename T, int ORDER>
__device__ __forceinline__ T d2_framed(const T* X, int p, int s, int i, int n, T uc, int w) {
    const bool nlo = (w & 1) != 0, nhi = (w & 2) != 0;
    T l1 = X[p - s], r1 = X[p + s];
    if (i == 0 && nlo) l1 = r1;
    if (i == n - 1 && nhi) r1 = l1;
    if (ORDER == 2) return l1 + r1 - T(2) * uc;
    T l2 = X[p - 2 * s], r2 = X[p + 2 * s];
    if (i == 0) l2 = nlo ? r2 : -uc;
    else if (i == 1 && nlo) l2 = uc;
    if (i == n - 1) r2 = nhi ? X[p - 2 * s] : -uc;
    else if (i == n - 2 && nhi) r2 = uc;
    return T(16) * (l1 + r1) - (l2 + r2) - T(30) * uc;
}

template <typename T, int ORDER>
__device__ __forceinline__ T axis_coef(double ih2) {
    return ORDER == 2 ? (T)ih2 : (T)(ih2 / 12.0);
}

// L_h u at point c = (i, j, k).  WALLS = false compiles the Dirichlet-only
// closure (g.wall is then ignored and must be 0).
template <typename T, int ORDER, int DIM, bool WALLS = true>
__device__ __forceinline__ T lap_at(const T* __restrict__ u, int64_t c, int i, int j, int k, const Geo& g, T uc) {
    const int w = WALLS ? g.wall : 0;
    T s = d2_axis<T, ORDER>(u, c, i, g.nx, 1, uc, w & 3) * axis_coef<T, ORDER>(g.ihx2);
    s += d2_axis<T, ORDER>(u, c, j, g.ny, g.nx, uc, (w >> 2) & 3) * axis_coef<T, ORDER>(g.ihy2);
    if (DIM == 3)
        s += d2_axis<T, ORDER>(u, c, k, g.nz, (int64_t)g.nx * g.ny, uc, (w >> 4) & 3) *
             axis_coef<T, ORDER>(g.ihz2);
    return s;
}

// Diagonal entry of L along one axis (un-scaled): -2 for order 2; order 4:
// -30, plus 1 where a Dirichlet wall's odd-reflection ghost refers back to
// the point itself (i = 0 or n-1), minus 1 where a Neumann wall's even ghost
// does (i = 1 or n-2).
template <typename T, int ORDER>
__device__ __forceinline__ T ldiag_axis(int i, int n, int w = 0) {
    if (ORDER == 2) return T(-2);
    const bool nlo = (w & 1) != 0, nhi = (w & 2) != 0;
    T d = T(-30);
    if (i == 0 && !nlo) d += T(1);
    if (i == n - 1 && !nhi) d += T(1);
    if (i == 1 && nlo) d -= T(1);
    if (i == n - 2 && nhi) d -= T(1);
    return d;
}

// True when the box [x0 - h, x1 + h) x [y0 - h, y1 + h) x [z0 - h, z1 + h)
// comes within two points of a Neumann wall: only tiles that do need the
// wall closures; every other tile of a box with Neumann walls runs the
// Dirichlet-only code, which is exact away from those walls.
__device__ __forceinline__ bool near_neumann(const Geo& g, int x0, int x1, int y0, int y1, int z0, int z1, int h) {
    return ((g.wall & 1) && x0 - h <= 1) || ((g.wall & 2) && x1 + h >= g.nx - 2) ||
           ((g.wall & 4) && y0 - h <= 1) || ((g.wall & 8) && y1 + h >= g.ny - 2) ||
           ((g.wall & 16) && z0 - h <= 1) || ((g.wall & 32) && z1 + h >= g.nz - 2);
}

// True when the 2D box [x0 - h, x1 + h) x [y0 - h, y1 + h) lies inside the
// grid.  A tile staged with that halo then loads no point beyond a wall, and
// every point it relaxes (at most h - R layers beyond the tile) lies at least
// R points inside: no wall, ghost or boundary diagonal enters, so its kernel
// may drop those tests (a uniform branch per tile) and still compute every
// value by the same expression.
__device__ __forceinline__ bool tile_inside2d(const Geo& g, int x0, int x1, int y0, int y1, int h) {
    return x0 - h >= 0 && x1 + h <= g.nx && y0 - h >= 0 && y1 + h <= g.ny;
}

// Diagonal of M = I - a L_h at (i, j, k) for the wall bits `wall` (Geo::wall
// layout); kernels compiled for Dirichlet-only boxes pass a literal 0 so that
// the Neumann cases fold away.
template <typename T, int ORDER, int DIM>
__device__ __forceinline__ T mdiag_w(int i, int j, int k, const Geo& g, T a, int wall) {
    T l = ldiag_axis<T, ORDER>(i, g.nx, wall & 3) * axis_coef<T, ORDER>(g.ihx2) +
          ldiag_axis<T, ORDER>(j, g.ny, (wall >> 2) & 3) * axis_coef<T, ORDER>(g.ihy2);
    if (DIM == 3) l += ldiag_axis<T, ORDER>(k, g.nz, (wall >> 4) & 3) * axis_coef<T, ORDER>(g.ihz2);
    return T(1) - a * l;
}

template <typename T, int ORDER, int DIM, bool WALLS = true>
__device__ __forceinline__ T mdiag_at(int i, int j, int k, const Geo& g, T a) {
    return mdiag_w<T, ORDER, DIM>(i, j, k, g, a, WALLS ? g.wall : 0);
}

// Block-wide sum for 256 threads (4 wavefronts of 64): wavefront shuffles then
// LDS.  The order of additions is fixed, so results are bitwise reproducible.
// `tid` is the linear thread index within the block.
__device__ __forceinline__ double block_sum_256(double v, int tid) {
    __shared__ double red[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = tid & 63, wid = tid >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;  // valid in thread 0 only
}

// Sum of the kRedBlocks partials, the same value in every thread of a
// one-dimensional block of 256 threads.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p) {
    __shared__ double total;
    double v = 0.0;
    for (int t = threadIdx.x; t < kRedBlocks; t += 256) v += p[t];
    double r = block_sum_256(v, threadIdx.x);
    if (threadIdx.x == 0) total = r;
    __syncthreads();
    return total;
}

}  // namespace ew
