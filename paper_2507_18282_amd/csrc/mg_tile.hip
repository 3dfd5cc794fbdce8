// Multigrid kernels tiled through LDS for the implicit step matrix
// M = I - a L_h (a = dt^2/2):
//
//  * k_sweep_tile    one full red-black Gauss-Seidel sweep (red half-sweep,
//                    then black) in a single pass: read x and b once, write x
//                    once.  Optionally the prolongation + correction of the
//                    coarse-grid solution is applied while the tile is loaded,
//                    and optionally the incoming iterate is known to be zero.
//  * k_restrict_tile residual at the fine points of a tile computed once in
//                    LDS, then full-weighting restriction.
//  * k_coarse_vcycle every level from a given one down to the coarsest, in
//                    one workgroup, with all level arrays resident in LDS.
//
// The arithmetic of each red or black half-sweep is the same as the simple
// kernels in mg.hip: x_i + (b - M x)_i / M_ii with every neighbour taken from
// the values before that half-sweep.
#include <hip/hip_ext.h>
#include <type_traits>

#include "mg_tile.h"
#include "stencil_dev.h"

#define EW_RET_ON_ERR(x)                   \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

namespace ew {

// ---------------------------------------------------------------------------
// Tile shapes
// ---------------------------------------------------------------------------
template <int DIM> struct SweepTile;
template <> struct SweepTile<2> { static constexpr int TX = 64, TY = 32, TZ = 1; };
template <> struct SweepTile<3> { static constexpr int TX = 32, TY = 8, TZ = 8; };
template <int DIM> struct RestrictTile;
// (NT: threads per workgroup; 512 measured 5 % slower on the 2047^2 level)
template <> struct RestrictTile<2> { static constexpr int CX = 32, CY = 16, CZ = 1, NT = 256; };
template <> struct RestrictTile<3> { static constexpr int CX = 16, CY = 4, CZ = 4, NT = 256; };

constexpr int kTileThreads = 256;

// Coarse neighbours of fine index f along one axis: q = f - off (off = 1
// behind a Dirichlet low wall, where coarse I sits at fine 2I + 1; 0 behind a
// Neumann one, where it sits at 2I); q even -> coarse q/2, odd -> mean of
// (q-1)/2 and (q+1)/2; a neighbour beyond a Dirichlet wall is dropped (0).
__device__ __forceinline__ void interp_axis(int f, int nc, int off, int& c0, int& c1, double& w0, double& w1) {
    const int q = f - off;
    if (q >= 0 && !(q & 1)) {
        c0 = q >> 1; c1 = -1; w0 = 1.0; w1 = 0.0;
    } else {
        c0 = (q - 1) >> 1; c1 = c0 + 1; w0 = 0.5; w1 = 0.5;
        if (c1 >= nc) c1 = -1;
    }
}

// Multilinear interpolation of the coarse grid function at fine point (i,j,k);
// wall = the fine level's Neumann-wall bits.
template <typename T, int DIM>
__device__ __forceinline__ T prolong_at(const T* __restrict__ xc, const Geo& gc, int i, int j, int k, int wall) {
    int xi[2], yj[2], zk[2];
    double wx[2], wy[2], wz[2];
    interp_axis(i, gc.nx, (wall & 1) ? 0 : 1, xi[0], xi[1], wx[0], wx[1]);
    interp_axis(j, gc.ny, (wall & 4) ? 0 : 1, yj[0], yj[1], wy[0], wy[1]);
    if (DIM == 3) interp_axis(k, gc.nz, (wall & 16) ? 0 : 1, zk[0], zk[1], wz[0], wz[1]);
    else { zk[0] = 0; zk[1] = -1; wz[0] = 1.0; wz[1] = 0.0; }
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
    return v;
}

// Second difference along one axis of an LDS tile (un-scaled), where cells
// outside the domain hold 0 (the wall); the order-4 ghost beyond the wall is
// the odd reflection of the point itself when it is the first or last point.
// IN: the point lies at least two points inside the grid (no ghost).
template <typename T, int ORDER, bool IN = false>
__device__ __forceinline__ T d2_lds(const T* X, int p, int stride, int gi, int n, T uc) {
    const T l1 = X[p - stride], r1 = X[p + stride];
    if (ORDER == 2) return l1 + r1 - T(2) * uc;
    const T l2 = (!IN && gi == 0) ? -uc : X[p - 2 * stride];
    const T r2 = (!IN && gi == n - 1) ? -uc : X[p + 2 * stride];
    return T(16) * (l1 + r1) - (l2 + r2) - T(30) * uc;
}

// L_h at LDS cell p whose neighbours beyond a wall read 0: the wall closures
// of d2_framed (Dirichlet odd reflection, Neumann even reflection).  WALLS =
// false compiles the Dirichlet-only closure, which `walls` = false (a tile
// away from Neumann walls) also selects; IN (a point at least two points
// inside the grid) drops the ghost tests of that closure.
// The axis coefficients of L_h, formed once per kernel (each is a division).
template <typename T>
struct AxisCoefs {
    T x, y, z;
};
template <typename T, int ORDER>
__device__ __forceinline__ AxisCoefs<T> axis_coefs(const Geo& g) {
    return {axis_coef<T, ORDER>(g.ihx2), axis_coef<T, ORDER>(g.ihy2), axis_coef<T, ORDER>(g.ihz2)};
}

template <typename T, int ORDER, int DIM, bool WALLS, bool IN = false>
__device__ __forceinline__ T lap_lds(const T* X, int p, int sy, int sz, int gi, int gj, int gk, const Geo& g, T uc,
                                     const AxisCoefs<T>& k, bool walls = true) {
    if (IN || !WALLS || !walls) {
        T s = d2_lds<T, ORDER, IN>(X, p, 1, gi, g.nx, uc) * k.x;
        s += d2_lds<T, ORDER, IN>(X, p, sy, gj, g.ny, uc) * k.y;
        if (DIM == 3) s += d2_lds<T, ORDER, IN>(X, p, sz, gk, g.nz, uc) * k.z;
        return s;
    }
    T s = d2_framed<T, ORDER>(X, p, 1, gi, g.nx, uc, g.wall & 3) * k.x;
    s += d2_framed<T, ORDER>(X, p, sy, gj, g.ny, uc, (g.wall >> 2) & 3) * k.y;
    if (DIM == 3) s += d2_framed<T, ORDER>(X, p, sz, gk, g.nz, uc, (g.wall >> 4) & 3) * k.z;
    return s;
}

// ---------------------------------------------------------------------------
// One full red-black sweep per tile.
// ---------------------------------------------------------------------------
template <typename T, int ORDER, int DIM, bool ZERO_IN, bool PROLONG, bool WALLS, int TX, int TY, int TZ>
__global__ __launch_bounds__(kTileThreads) void k_sweep_tile(const T* __restrict__ xin, const T* __restrict__ xc,
                                                             const T* __restrict__ b, T bscale, T* __restrict__ xout,
                                                             Geo g, Geo gc, T a, T w) {
    constexpr int R = ORDER / 2;        // stencil radius
    constexpr int H = R + 1;            // red is relaxed on the tile plus one layer
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H, LZ = (DIM == 3) ? TZ + 2 * H : 1;
    constexpr int BX = TX + 2, BY = TY + 2, BZ = (DIM == 3) ? TZ + 2 : 1;
    constexpr int NRED = BX * BY * BZ;
    constexpr int RED_ITERS = (NRED + kTileThreads - 1) / kTileThreads;
    __shared__ T X[LX * LY * LZ];
    __shared__ T B[BX * BY * BZ];
    const int tid = threadIdx.x;
    const AxisCoefs<T> kc = axis_coefs<T, ORDER>(g);
    int bx, by, bz;
    xcd_block(bx, by, bz);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY, z0 = (DIM == 3) ? bz * TZ : 0;
    const bool nw = WALLS && near_neumann(g, x0, x0 + TX, y0, y0 + TY, z0, z0 + TZ, H);  // uniform per tile

    // Staging of x (tile + H, zero outside the domain) and b (tile + 1): every
    // global load of a thread is issued into registers before its first LDS
    // store, so the block waits for memory once.  The prolongation (coarse
    // values read through the cache) is added afterwards, in LDS.
    constexpr int NX = LX * LY * LZ, NB = BX * BY * BZ;
    constexpr int IX = (NX + kTileThreads - 1) / kTileThreads, IB = (NB + kTileThreads - 1) / kTileThreads;
    T xv[IX], bv[IB];
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kTileThreads;
        T v = T(0);
        if (!ZERO_IN && q < NX) {
            const int lx = q % LX, ly = (q / LX) % LY, lz = q / (LX * LY);
            const int gi = x0 - H + lx, gj = y0 - H + ly, gk = (DIM == 3) ? z0 - H + lz : 0;
            if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny && gk >= 0 && gk < g.nz) v = xin[lin(g, gi, gj, gk)];
        }
        xv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * kTileThreads;
        T v = T(0);
        if (q < NB) {
            const int bx = q % BX, by = (q / BX) % BY, bz = q / (BX * BY);
            const int gi = x0 - 1 + bx, gj = y0 - 1 + by, gk = (DIM == 3) ? z0 - 1 + bz : 0;
            if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny && gk >= 0 && gk < g.nz) v = b[lin(g, gi, gj, gk)];
        }
        bv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kTileThreads;
        if (q < NX) X[q] = xv[t];
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * kTileThreads;
        if (q < NB) B[q] = bscale * bv[t];
    }
    if (PROLONG) {
        // each thread updates only the cells it stored itself: no barrier needed before
        for (int q = tid; q < NX; q += kTileThreads) {
            const int lx = q % LX, ly = (q / LX) % LY, lz = q / (LX * LY);
            const int gi = x0 - H + lx, gj = y0 - H + ly, gk = (DIM == 3) ? z0 - H + lz : 0;
            if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny && gk >= 0 && gk < g.nz)
                X[q] += prolong_at<T, DIM>(xc, gc, gi, gj, gk, WALLS ? g.wall : 0);
        }
    }
    __syncthreads();

    // red half-sweep on tile + 1 layer: new values to registers first (order 4
    // couples red points to red points), then into LDS
    T rv[RED_ITERS];
    int rp[RED_ITERS];
#pragma unroll
    for (int t = 0; t < RED_ITERS; ++t) {
        rp[t] = -1;
        const int q = tid + t * kTileThreads;
        if (q >= NRED) continue;
        const int bx = q % BX, by = (q / BX) % BY, bz = q / (BX * BY);
        const int gi = x0 - 1 + bx, gj = y0 - 1 + by, gk = (DIM == 3) ? z0 - 1 + bz : 0;
        if (gi < 0 || gi >= g.nx || gj < 0 || gj >= g.ny || gk < 0 || gk >= g.nz) continue;
        if (((gi + gj + gk) & 1) != 0) continue;
        const int p = (bx + H - 1) + LX * ((by + H - 1) + LY * ((DIM == 3) ? (bz + H - 1) : 0));
        const T uc = X[p];
        const T lap = lap_lds<T, ORDER, DIM, WALLS>(X, p, LX, LX * LY, gi, gj, gk, g, uc, kc, nw);
        const T r = B[q] - (uc - a * lap);
        rv[t] = uc + (w * r) / mdiag_w<T, ORDER, DIM>(gi, gj, gk, g, a, nw ? g.wall : 0);
        rp[t] = p;
    }
    if (ORDER == 4) __syncthreads();  // same-colour neighbours are read old (order 4 only)
#pragma unroll
    for (int t = 0; t < RED_ITERS; ++t)
        if (rp[t] >= 0) X[rp[t]] = rv[t];
    __syncthreads();

    // black half-sweep on the tile, written straight to global memory
    for (int q = tid; q < TX * TY * TZ; q += kTileThreads) {
        const int tx = q % TX, ty = (q / TX) % TY, tz = q / (TX * TY);
        const int gi = x0 + tx, gj = y0 + ty, gk = z0 + tz;
        if (gi >= g.nx || gj >= g.ny || gk >= g.nz) continue;
        const int p = (tx + H) + LX * ((ty + H) + LY * ((DIM == 3) ? (tz + H) : 0));
        const T uc = X[p];
        T out = uc;
        if (((gi + gj + gk) & 1) == 1) {
            const T lap = lap_lds<T, ORDER, DIM, WALLS>(X, p, LX, LX * LY, gi, gj, gk, g, uc, kc, nw);
            const int qb = (tx + 1) + BX * ((ty + 1) + BY * ((DIM == 3) ? (tz + 1) : 0));
            const T r = B[qb] - (uc - a * lap);
            out = uc + (w * r) / mdiag_w<T, ORDER, DIM>(gi, gj, gk, g, a, nw ? g.wall : 0);
        }
        xout[lin(g, gi, gj, gk)] = out;
    }
}

// ---------------------------------------------------------------------------
// One full red-black sweep of an order-2 3D level without Neumann walls, by
// marching a 64 x TY column tile through a chunk of `chunk` planes.  Planes of x
// (xy halo 2) and b (xy halo 1) pass through LDS rings of 5 and 3 slots.
// Step k relaxes the red points of plane k on the tile plus one xy layer (its
// z-neighbours on planes k +- 1 are black and still old), then the black
// points of plane k-1 on the tile (all their neighbours are red and final),
// and writes plane k-1.  The chunk starts one plane early: the red points of
// plane z0-1 are recomputed from old values, as the chunk below computes
// them (x is read from xin and written to xout, never in place).  The loads
// of the next planes are issued one step ahead, into registers.  Same
// arithmetic as k_sweep_tile except that the weight and the constant diagonal
// enter as one reciprocal.
//
// With PROLONG the trilinear interpolation of the coarse solution xc (the
// prolongation of the V-cycle's coarse-grid correction) is added to every x
// plane as it enters the ring: the coarse values under the tile are first
// combined along z for that fine plane (Cz, two coarse planes, staged one
// step ahead in a double-buffered LDS slot), then interpolated in x and y
// from LDS.
// ---------------------------------------------------------------------------
template <typename T, bool ZERO_IN, bool PROLONG, int TY>
__global__ __launch_bounds__(kTileThreads) void k_sweep_z3d(const T* __restrict__ xin, const T* __restrict__ xc,
                                                            const T* __restrict__ b, T bscale, T* __restrict__ xout,
                                                            Geo g, Geo gc, T a, T inv_diag, int chunk) {
    constexpr int TX = 64;
    constexpr int LX = TX + 4, LY = TY + 4, NXP = LX * LY;  // x plane, halo 2
    constexpr int BX = TX + 2, BY = TY + 2, NBP = BX * BY;  // b plane, halo 1
    constexpr int IXP = (NXP + kTileThreads - 1) / kTileThreads, IBP = (NBP + kTileThreads - 1) / kTileThreads;
    constexpr int NRP = (BY + 7) / 8;                       // red rows per lane
    // coarse cells under an x plane: columns x0/2 - 2 .. x0/2 + 32, rows
    // y0/2 - 2 .. y0/2 + TY/2 (fine f interpolates coarse (f-1)/2 rounded down and up)
    constexpr int CXW = 36, CYW = TY / 2 + 3, NCP = CXW * CYW;
    constexpr int ICP = PROLONG ? (NCP + kTileThreads - 1) / kTileThreads : 1;
    static_assert(TY % 8 == 0, "black rows are handed out 8 per pass");
    __shared__ T X[5][NXP];
    __shared__ T B[3][NBP];
    __shared__ T CZS[2][PROLONG ? NCP : 1];
    const int tid = threadIdx.x;
    int bx, by, bz;
    xcd_block(bx, by, bz);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * chunk;
    const int z1 = min(z0 + chunk, g.nz);  // planes written: [z0, z1)
    const int64_t plane = (int64_t)g.nx * g.ny;
    const T cx = (T)g.ihx2, cy = (T)g.ihy2, cz = (T)g.ihz2;
    auto xslot = [](int k) { return (k + 5) % 5; };  // k >= -2
    auto bslot = [](int k) { return (k + 3) % 3; };
    const int ccx0 = (x0 >> 1) - 2, ccy0 = (y0 >> 1) - 2;
    const int64_t cplane = (int64_t)gc.nx * gc.ny;

    // registers of the planes in flight (issuing the loads two steps ahead,
    // in two register sets, measured slower)
    struct Regs {
        T x[IXP], b[IBP], c[ICP];
    };
    Regs RA;
    // coarse values for fine plane f combined along z: f interpolates coarse
    // plane (f-1)/2 if f-1 is even, else the mean of (f-2)/2 and f/2 (planes
    // beyond the coarse grid are the zero wall)
    auto load_cz = [&](T(&cv)[ICP], int f) {
#pragma unroll
        for (int t = 0; t < ICP; ++t) {
            const int q = tid + t * kTileThreads;
            T v = T(0);
            if (PROLONG && q < NCP && f >= 0 && f < g.nz) {
                const int cy = q / CXW, cxx = q - cy * CXW;
                const int ic = ccx0 + cxx, jc = ccy0 + cy;
                if (ic >= 0 && ic < gc.nx && jc >= 0 && jc < gc.ny) {
                    const int qz = f - 1;
                    const int64_t o = (int64_t)jc * gc.nx + ic;
                    if (!(qz & 1)) {
                        v = xc[(qz >> 1) * cplane + o];
                    } else {
                        const int ka = (qz - 1) >> 1, kb2 = ka + 1;
                        const T va = ka >= 0 ? xc[ka * cplane + o] : T(0);
                        const T vb = kb2 < gc.nz ? xc[kb2 * cplane + o] : T(0);
                        v = T(0.5) * va + T(0.5) * vb;
                    }
                }
            }
            cv[t] = v;
        }
    };
    auto store_cz = [&](const T(&cv)[ICP], int f) {
        T* dst = CZS[f & 1];
#pragma unroll
        for (int t = 0; t < ICP; ++t) {
            const int q = tid + t * kTileThreads;
            if (PROLONG && q < NCP) dst[q] = cv[t];
        }
    };
    // global loads of x plane k (tile + 2, zero outside the domain) into xv
    auto load_x = [&](T(&xv)[IXP], int k) {
#pragma unroll
        for (int t = 0; t < IXP; ++t) {
            const int q = tid + t * kTileThreads;
            T v = T(0);
            if (!ZERO_IN && q < NXP && k >= 0 && k < g.nz) {
                const int ly = q / LX, lx = q - ly * LX;
                const int gi = x0 - 2 + lx, gj = y0 - 2 + ly;
                if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny) v = xin[k * plane + (int64_t)gj * g.nx + gi];
            }
            xv[t] = v;
        }
    };
    auto load_b = [&](T(&bv)[IBP], int k) {
#pragma unroll
        for (int t = 0; t < IBP; ++t) {
            const int q = tid + t * kTileThreads;
            T v = T(0);
            if (q < NBP && k >= 0 && k < g.nz) {
                const int ly = q / BX, lx = q - ly * BX;
                const int gi = x0 - 1 + lx, gj = y0 - 1 + ly;
                if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny) v = b[k * plane + (int64_t)gj * g.nx + gi];
            }
            bv[t] = v;
        }
    };
    // x plane k into its slot, plus the bilinear interpolation of Cz(k) (in
    // CZS[k & 1]) at the cells inside the domain with PROLONG
    auto store_x = [&](const T(&xv)[IXP], int k) {
        T* dst = X[xslot(k)];
        const T* cz = CZS[k & 1];
#pragma unroll
        for (int t = 0; t < IXP; ++t) {
            const int q = tid + t * kTileThreads;
            if (q >= NXP) continue;
            T v = xv[t];
            if (PROLONG && k >= 0 && k < g.nz) {
                const int ly = q / LX, lx = q - ly * LX;
                const int gi = x0 - 2 + lx, gj = y0 - 2 + ly;
                if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny) {
                    const int qi = gi - 1, qj = gj - 1;
                    const int ia = (qi >> 1) - ccx0, ib = ((qi + 1) >> 1) - ccx0;
                    const int ja = (qj >> 1) - ccy0, jb = ((qj + 1) >> 1) - ccy0;
                    const T wia = (qi & 1) ? T(0.5) : T(1), wib = (qi & 1) ? T(0.5) : T(0);
                    const T wja = (qj & 1) ? T(0.5) : T(1), wjb = (qj & 1) ? T(0.5) : T(0);
                    const T rowa = wia * cz[ja * CXW + ia] + wib * cz[ja * CXW + ib];
                    const T rowb = wia * cz[jb * CXW + ia] + wib * cz[jb * CXW + ib];
                    v += wja * rowa + wjb * rowb;
                }
            }
            dst[q] = v;
        }
    };
    auto store_b = [&](const T(&bv)[IBP], int k) {
        T* dst = B[bslot(k)];
#pragma unroll
        for (int t = 0; t < IBP; ++t) {
            const int q = tid + t * kTileThreads;
            if (q < NBP) dst[q] = bscale * bv[t];
        }
    };
    // relaxed value of LDS cell p of plane k (slots of k-1, k, k+1 given)
    auto relax = [&](const T* Xm, const T* X0, const T* Xp, int p, T bval) -> T {
        const T uc = X0[p];
        T s = (X0[p - 1] + X0[p + 1] - T(2) * uc) * cx;
        s += (X0[p - LX] + X0[p + LX] - T(2) * uc) * cy;
        s += (Xm[p] + Xp[p] - T(2) * uc) * cz;
        const T r = bval - (uc - a * s);
        return uc + r * inv_diag;
    };

    // prologue: x planes z0-2 and z0-1 in the ring (with PROLONG after Cz of
    // those planes, and Cz(z0) in its slot), then the loads of x plane z0, b
    // plane z0-1 and Cz(z0+1) in flight (step k stores x plane k+1, b plane k
    // and Cz(k+2), and issues the loads of the next step)
    if (PROLONG) {
        load_cz(RA.c, z0 - 2);
        store_cz(RA.c, z0 - 2);
        load_cz(RA.c, z0 - 1);
        store_cz(RA.c, z0 - 1);
        __syncthreads();
    }
    load_x(RA.x, z0 - 2);
    store_x(RA.x, z0 - 2);
    load_x(RA.x, z0 - 1);
    store_x(RA.x, z0 - 1);
    if (PROLONG) {
        __syncthreads();  // slot (z0-2) & 1 is read above; Cz(z0) replaces it
        load_cz(RA.c, z0);
        store_cz(RA.c, z0);
        __syncthreads();
        load_cz(RA.c, z0 + 1);
    }
    load_x(RA.x, z0);
    load_b(RA.b, z0 - 1);

    // 8 rows per pass, 32 lanes per row; the lanes of a wavefront alternate
    // between its two rows, whose points of one colour sit in columns of
    // opposite parity (LX and BX are even), so consecutive lanes read
    // distinct LDS banks
    static_assert(LX % 2 == 0 && BX % 2 == 0, "paired rows must start on opposite column parities");
    const int rowsel = ((tid >> 6) << 1) | (tid & 1), m = (tid >> 1) & 31;
    auto step = [&](int k, Regs& R) {
        // planes k+1 (x) and k (b) arrive; issue the loads of the next step
        store_x(R.x, k + 1);
        store_b(R.b, k);
        if (PROLONG) store_cz(R.c, k + 2);  // into the slot of Cz(k), last read at step k-1
        if (k < z1) {
            load_x(R.x, k + 2);
            load_b(R.b, k + 1);
            if (PROLONG) load_cz(R.c, k + 3);
        }
        __syncthreads();
        // red points of plane k on the tile plus one xy layer
        if (k >= 0 && k < g.nz) {
            const T* Xm = X[xslot(k - 1)];
            T* X0 = X[xslot(k)];
            const T* Xp = X[xslot(k + 1)];
            const T* Bk = B[bslot(k)];
#pragma unroll
            for (int t = 0; t < NRP; ++t) {
                const int ry = rowsel + 8 * t;
                if (ry >= BY) continue;
                const int gj = y0 - 1 + ry;
                const int c = 2 * m + ((gj + k) & 1);  // tile column of the red point (x0 is even)
                const int gi = x0 + c;
                if (gj < 0 || gj >= g.ny || gi >= g.nx) continue;
                const int p = (ry + 1) * LX + c + 2;
                X0[p] = relax(Xm, X0, Xp, p, Bk[ry * BX + c + 1]);
            }
            if (tid < BY) {  // the red point of each row in tile column -1 or 64
                const int ry = tid, gj = y0 - 1 + ry;
                const int c = ((gj + k) & 1) ? -1 : 64;
                const int gi = x0 + c;
                if (gj >= 0 && gj < g.ny && gi >= 0 && gi < g.nx) {
                    const int p = (ry + 1) * LX + c + 2;
                    X0[p] = relax(Xm, X0, Xp, p, Bk[ry * BX + c + 1]);
                }
            }
        }
        __syncthreads();
        // black points of plane k-1 on the tile; each lane writes its black
        // point and the red point beside it
        const int kb = k - 1;
        if (kb >= z0 && kb < z1) {
            const T* Xm = X[xslot(kb - 1)];
            const T* X0 = X[xslot(kb)];
            const T* Xp = X[xslot(kb + 1)];
            const T* Bk = B[bslot(kb)];
#pragma unroll
            for (int t = 0; t < TY / 8; ++t) {
                const int ty = rowsel + 8 * t;
                const int gj = y0 + ty;
                if (gj >= g.ny) continue;
                const int cb = 2 * m + ((gj + kb + 1) & 1), cr = cb ^ 1;
                const int gib = x0 + cb, gir = x0 + cr;
                T* row = xout + kb * plane + (int64_t)gj * g.nx;
                const int pb = (ty + 2) * LX + cb + 2;
                if (gib < g.nx) row[gib] = relax(Xm, X0, Xp, pb, Bk[(ty + 1) * BX + cb + 1]);
                if (gir < g.nx) row[gir] = X0[(ty + 2) * LX + cr + 2];
            }
        }
        // no barrier here: the next step stores into the slots of planes
        // k-3 (x) and k+1 (b), which the black phase does not read
    };
    for (int k = z0 - 1; k <= z1; ++k) step(k, RA);
}

// ---------------------------------------------------------------------------
// Residual norm per tile: x staged with a halo of R (zero outside the domain,
// the wall closures of lap_lds), r = bscale b - M x at the tile's points,
// optionally stored (converted to TR), and the tile's sum of r^2 written to
// tile_partial[tile] (tiles in their logical order).  k_fold_partials then
// sums the tile partials into the kRedBlocks partials the host reads, each in
// a fixed order.
// ---------------------------------------------------------------------------
template <int DIM> struct ResTile;
template <> struct ResTile<2> { static constexpr int TX = 64, TY = 8, TZ = 1; };
template <> struct ResTile<3> { static constexpr int TX = 32, TY = 8, TZ = 4; };

int64_t residual_tiles(const Geo& g) {
    if (g.dim == 2)
        return (int64_t)((g.nx + ResTile<2>::TX - 1) / ResTile<2>::TX) * ((g.ny + ResTile<2>::TY - 1) / ResTile<2>::TY);
    return (int64_t)((g.nx + ResTile<3>::TX - 1) / ResTile<3>::TX) * ((g.ny + ResTile<3>::TY - 1) / ResTile<3>::TY) *
           ((g.nz + ResTile<3>::TZ - 1) / ResTile<3>::TZ);
}

// One tile of k_residual_tile; IN: a 2D tile whose staged halo lies inside
// the grid (tile_inside2d), so no load, point or ghost needs a test.
template <typename T, typename TR, int ORDER, int DIM, bool WALLS, bool IN>
__device__ __forceinline__ double residual_tile_body(const T* __restrict__ x, const T* __restrict__ b, T bscale,
                                                     const Geo& g, T a, TR* __restrict__ r_out, T* X, int tid,
                                                     int x0, int y0, int z0, bool nw) {
    constexpr int TX = ResTile<DIM>::TX, TY = ResTile<DIM>::TY, TZ = ResTile<DIM>::TZ;
    constexpr int R = ORDER / 2;
    constexpr int LX = TX + 2 * R, LY = TY + 2 * R, LZ = (DIM == 3) ? TZ + 2 * R : 1;
    constexpr int NX = LX * LY * LZ, NP = TX * TY * TZ;
    constexpr int IX = (NX + kTileThreads - 1) / kTileThreads, IP = NP / kTileThreads;
    const AxisCoefs<T> kc = axis_coefs<T, ORDER>(g);
    // every global load of a thread is issued before the first LDS store
    T xv[IX], bv[IP];
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kTileThreads;
        T v = T(0);
        if (q < NX) {
            const int lx = q % LX, ly = (q / LX) % LY, lz = q / (LX * LY);
            const int gi = x0 - R + lx, gj = y0 - R + ly, gk = (DIM == 3) ? z0 - R + lz : 0;
            if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny && gk >= 0 && gk < g.nz))
                v = x[lin(g, gi, gj, gk)];
        }
        xv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IP; ++t) {
        const int q = tid + t * kTileThreads;
        const int gi = x0 + q % TX, gj = y0 + (q / TX) % TY, gk = z0 + q / (TX * TY);
        bv[t] = (IN || (gi < g.nx && gj < g.ny && gk < g.nz)) ? b[lin(g, gi, gj, gk)] : T(0);
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kTileThreads;
        if (q < NX) X[q] = xv[t];
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < IP; ++t) {
        const int q = tid + t * kTileThreads;
        const int tx = q % TX, ty = (q / TX) % TY, tz = q / (TX * TY);
        const int gi = x0 + tx, gj = y0 + ty, gk = z0 + tz;
        if (!IN && (gi >= g.nx || gj >= g.ny || gk >= g.nz)) continue;
        const int p = (tx + R) + LX * ((ty + R) + LY * ((DIM == 3) ? (tz + R) : 0));
        const T uc = X[p];
        const T r = bscale * bv[t] -
                    (uc - a * lap_lds<T, ORDER, DIM, WALLS, IN>(X, p, LX, LX * LY, gi, gj, gk, g, uc, kc, nw));
        if (r_out) r_out[lin(g, gi, gj, gk)] = (TR)r;
        acc += (double)r * (double)r;
    }
    return acc;
}

template <typename T, typename TR, int ORDER, int DIM, bool WALLS>
__global__ __launch_bounds__(kTileThreads) void k_residual_tile(const T* __restrict__ x, const T* __restrict__ b,
                                                                T bscale, Geo g, T a, double* __restrict__ tile_partial,
                                                                TR* __restrict__ r_out) {
    constexpr int TX = ResTile<DIM>::TX, TY = ResTile<DIM>::TY, TZ = ResTile<DIM>::TZ;
    constexpr int R = ORDER / 2;
    constexpr int LX = TX + 2 * R, LY = TY + 2 * R, LZ = (DIM == 3) ? TZ + 2 * R : 1;
    static_assert((TX * TY * TZ) % kTileThreads == 0, "whole points per thread");
    __shared__ T X[LX * LY * LZ];
    const int tid = threadIdx.x;
    int bx, by, bz;
    xcd_block(bx, by, bz);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY, z0 = (DIM == 3) ? bz * TZ : 0;
    const bool nw = WALLS && near_neumann(g, x0, x0 + TX, y0, y0 + TY, z0, z0 + TZ, R);  // uniform per tile
    double acc;
    if constexpr (DIM == 2) {
        if (!nw && tile_inside2d(g, x0, x0 + TX, y0, y0 + TY, R))
            acc = residual_tile_body<T, TR, ORDER, DIM, WALLS, true>(x, b, bscale, g, a, r_out, X, tid, x0, y0, z0, nw);
        else
            acc = residual_tile_body<T, TR, ORDER, DIM, WALLS, false>(x, b, bscale, g, a, r_out, X, tid, x0, y0, z0, nw);
    } else {
        acc = residual_tile_body<T, TR, ORDER, DIM, WALLS, false>(x, b, bscale, g, a, r_out, X, tid, x0, y0, z0, nw);
    }
    const double s = block_sum_256(acc, tid);
    if (tid == 0) tile_partial[bx + gridDim.x * (by + gridDim.y * bz)] = s;
}

__global__ __launch_bounds__(kRedBlocks) void k_fold_partials(const double* __restrict__ tile_partial, int ntiles,
                                                              double* __restrict__ partial) {
    double s = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += kRedBlocks) s += tile_partial[i];
    partial[threadIdx.x] = s;
}

template <typename T, typename TR>
hipError_t launch_residual_tile(const T* x, const T* b, double bscale, const Geo& g, int order, double a,
                                double* tile_partial, double* partial, TR* r_out, hipStream_t s) {
    const T bs = (T)bscale, aa = (T)a;
#define EW_RT(O, D)                                                                                            \
    do {                                                                                                       \
        constexpr int TX = ResTile<D>::TX, TY = ResTile<D>::TY, TZ = ResTile<D>::TZ;                           \
        dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, D == 3 ? (g.nz + TZ - 1) / TZ : 1);              \
        if (g.wall)                                                                                            \
            k_residual_tile<T, TR, O, D, true><<<grid, kTileThreads, 0, s>>>(x, b, bs, g, aa, tile_partial, r_out); \
        else                                                                                                   \
            k_residual_tile<T, TR, O, D, false><<<grid, kTileThreads, 0, s>>>(x, b, bs, g, aa, tile_partial, r_out); \
    } while (0)
    if (g.dim == 2) {
        if (order == 2) EW_RT(2, 2); else EW_RT(4, 2);
    } else {
        if (order == 2) EW_RT(2, 3); else EW_RT(4, 3);
    }
#undef EW_RT
    EW_RET_ON_ERR(hipGetLastError());
    k_fold_partials<<<1, kRedBlocks, 0, s>>>(tile_partial, (int)residual_tiles(g), partial);
    return hipGetLastError();
}
template hipError_t launch_residual_tile<double, double>(const double*, const double*, double, const Geo&, int, double,
                                                         double*, double*, double*, hipStream_t);
template hipError_t launch_residual_tile<double, float>(const double*, const double*, double, const Geo&, int, double,
                                                        double*, double*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// Residual + full-weighting restriction per coarse tile.
// ---------------------------------------------------------------------------
// One coarse tile of k_restrict_tile; IN: a 2D tile whose fine region and
// stencil reach lie inside the grid (tile_inside2d), so no load, point or
// ghost needs a test.
template <typename T, int ORDER, int DIM, int CY, bool WALLS, bool IN, int NT>
__device__ __forceinline__ void restrict_tile_body(const T* __restrict__ x, const T* __restrict__ b, T bscale,
                                                   const Geo& gf, T a, T* __restrict__ bc, const Geo& gc, T* X, T* Rf,
                                                   int tid, int cx0, int cy0, int cz0, int fx0, int fy0, int fz0,
                                                   bool nw) {
    constexpr int CX = RestrictTile<DIM>::CX, CZ = RestrictTile<DIM>::CZ;
    constexpr int R = ORDER / 2;
    constexpr int FX = 2 * CX + 1, FY = 2 * CY + 1, FZ = (DIM == 3) ? 2 * CZ + 1 : 1;
    constexpr int LX = FX + 2 * R, LY = FY + 2 * R, LZ = (DIM == 3) ? FZ + 2 * R : 1;
    const AxisCoefs<T> kc = axis_coefs<T, ORDER>(gf);
    // Staging as in the sweep: x (region + R) and b (region) go to registers
    // with every load issued before the first use.
    constexpr int NX = LX * LY * LZ, NF = FX * FY * FZ;
    constexpr int IX = (NX + NT - 1) / NT, IF = (NF + NT - 1) / NT;
    T xv[IX], bv[IF];
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * NT;
        T v = T(0);
        if (q < NX) {
            const int lx = q % LX, ly = (q / LX) % LY, lz = q / (LX * LY);
            const int gi = fx0 - R + lx, gj = fy0 - R + ly, gk = (DIM == 3) ? fz0 - R + lz : 0;
            if (IN || (gi >= 0 && gi < gf.nx && gj >= 0 && gj < gf.ny && gk >= 0 && gk < gf.nz))
                v = x[lin(gf, gi, gj, gk)];
        }
        xv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IF; ++t) {
        const int q = tid + t * NT;
        T v = T(0);
        if (q < NF) {
            const int fx = q % FX, fy = (q / FX) % FY, fz = q / (FX * FY);
            const int gi = fx0 + fx, gj = fy0 + fy, gk = fz0 + fz;
            // (a region starts below index 0 only when shifted)
            if (IN || ((!WALLS || (gi >= 0 && gj >= 0 && gk >= 0)) && gi < gf.nx && gj < gf.ny && gk < gf.nz))
                v = b[lin(gf, gi, gj, gk)];
        }
        bv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * NT;
        if (q < NX) X[q] = xv[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < IF; ++t) {
        const int q = tid + t * NT;
        if (q >= NF) continue;
        const int fx = q % FX, fy = (q / FX) % FY, fz = q / (FX * FY);
        const int gi = fx0 + fx, gj = fy0 + fy, gk = fz0 + fz;
        T r = T(0);
        if (IN || ((!WALLS || (gi >= 0 && gj >= 0 && gk >= 0)) && gi < gf.nx && gj < gf.ny && gk < gf.nz)) {
            const int p = (fx + R) + LX * ((fy + R) + LY * ((DIM == 3) ? (fz + R) : 0));
            const T uc = X[p];
            r = bscale * bv[t] -
                (uc - a * lap_lds<T, ORDER, DIM, WALLS, IN>(X, p, LX, LX * LY, gi, gj, gk, gf, uc, kc, nw));
        }
        Rf[q] = r;
    }
    __syncthreads();
    if (!IN && nw) {
        // region cells beyond a Neumann wall take the residual of their even
        // mirror inside the box (only in-range cells are read here)
        for (int q = tid; q < NF; q += NT) {
            const int fx = q % FX, fy = (q / FX) % FY, fz = q / (FX * FY);
            int gi = fx0 + fx, gj = fy0 + fy, gk = fz0 + fz;
            const bool out = gi < 0 || gi >= gf.nx || gj < 0 || gj >= gf.ny || gk < 0 || gk >= gf.nz;
            if (!out) continue;
            if (gi < 0 && (gf.wall & 1)) gi = -gi;
            if (gi >= gf.nx && (gf.wall & 2)) gi = 2 * (gf.nx - 1) - gi;
            if (gj < 0 && (gf.wall & 4)) gj = -gj;
            if (gj >= gf.ny && (gf.wall & 8)) gj = 2 * (gf.ny - 1) - gj;
            if (DIM == 3 && gk < 0 && (gf.wall & 16)) gk = -gk;
            if (DIM == 3 && gk >= gf.nz && (gf.wall & 32)) gk = 2 * (gf.nz - 1) - gk;
            if (gi < 0 || gi >= gf.nx || gj < 0 || gj >= gf.ny || gk < 0 || gk >= gf.nz)
                continue;  // beyond a Dirichlet wall: stays 0
            Rf[q] = Rf[(gi - fx0) + FX * ((gj - fy0) + FY * (gk - fz0))];
        }
        __syncthreads();
    }
    for (int q = tid; q < CX * CY * CZ; q += NT) {
        const int cx = q % CX, cy = (q / CX) % CY, cz = q / (CX * CY);
        const int ic = cx0 + cx, jc = cy0 + cy, kc = cz0 + cz;
        if (ic >= gc.nx || jc >= gc.ny || kc >= gc.nz) continue;
        const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = (DIM == 3) ? 2 * cz + 1 : 0;
        T sum = T(0);
        if (DIM == 2) {
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy) {
                T row = T(0);
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox)
                    row += (ox == 0 ? T(0.5) : T(0.25)) * Rf[(fx + ox) + FX * (fy + oy)];
                sum += (oy == 0 ? T(0.5) : T(0.25)) * row;
            }
        } else {
#pragma unroll
            for (int oz = -1; oz <= 1; ++oz) {
                T plane = T(0);
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy) {
                    T row = T(0);
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox)
                        row += (ox == 0 ? T(0.5) : T(0.25)) * Rf[(fx + ox) + FX * ((fy + oy) + FY * (fz + oz))];
                    plane += (oy == 0 ? T(0.5) : T(0.25)) * row;
                }
                sum += (oz == 0 ? T(0.5) : T(0.25)) * plane;
            }
        }
        bc[lin(gc, ic, jc, kc)] = sum;
    }
}

template <typename T, int ORDER, int DIM, int CY, bool WALLS, int NT>
__global__ __launch_bounds__(NT) void k_restrict_tile(const T* __restrict__ x, const T* __restrict__ b,
                                                                T bscale, Geo gf, T a, T* __restrict__ bc, Geo gc) {
    constexpr int CX = RestrictTile<DIM>::CX, CZ = RestrictTile<DIM>::CZ;
    constexpr int R = ORDER / 2;
    constexpr int FX = 2 * CX + 1, FY = 2 * CY + 1, FZ = (DIM == 3) ? 2 * CZ + 1 : 1;
    constexpr int LX = FX + 2 * R, LY = FY + 2 * R, LZ = (DIM == 3) ? FZ + 2 * R : 1;
    __shared__ T X[LX * LY * LZ];
    __shared__ T Rf[FX * FY * FZ];
    const int tid = threadIdx.x;
    int bx, by, bz;
    xcd_block(bx, by, bz);  // XCD-contiguous bands of tiles
    const int cx0 = bx * CX, cy0 = by * CY, cz0 = (DIM == 3) ? bz * CZ : 0;
    // first fine point of the region: fine centre of coarse I is 2I + 1 behind
    // a Dirichlet low wall, 2I behind a Neumann one (WALLS, 2D)
    const int sx = (WALLS && (gf.wall & 1)) ? -1 : 0, sy = (WALLS && (gf.wall & 4)) ? -1 : 0;
    const int sz = (WALLS && DIM == 3 && (gf.wall & 16)) ? -1 : 0;
    const int fx0 = 2 * cx0 + sx, fy0 = 2 * cy0 + sy, fz0 = (DIM == 3) ? 2 * cz0 + sz : 0;
    // the region and its stencil reach: fine points [f0 - R, f0 + F + R) per direction
    const bool nw = WALLS && near_neumann(gf, fx0, fx0 + FX, fy0, fy0 + FY, fz0, fz0 + FZ, R);  // uniform per tile
    if constexpr (DIM == 2) {
        if (!nw && tile_inside2d(gf, fx0, fx0 + FX, fy0, fy0 + FY, R)) {
            restrict_tile_body<T, ORDER, DIM, CY, WALLS, true, NT>(x, b, bscale, gf, a, bc, gc, X, Rf, tid, cx0, cy0, cz0,
                                                               fx0, fy0, fz0, nw);
            return;
        }
    }
    restrict_tile_body<T, ORDER, DIM, CY, WALLS, false, NT>(x, b, bscale, gf, a, bc, gc, X, Rf, tid, cx0, cy0, cz0, fx0,
                                                        fy0, fz0, nw);
}

// ---------------------------------------------------------------------------
// Coarse levels in one workgroup: V(nu1, nu2) from level 0 of `c` (whose
// right-hand side is read from global memory) down to the coarsest, all level
// arrays in dynamic LDS.  Each level is stored with a zero halo of two cells
// (the wall, and the cell beyond it that only the order-4 ghost would use, which
// is handled explicitly), so stencils need no bounds tests.  Threads own fixed
// columns (2D: i = tid % 64, rows j = tid / 64 + 16 t; 3D: i = tid % 16,
// j = tid / 16 % 16, planes k = tid / 256 + 4 t), so no index divisions occur.
// The result on level 0 is written to x_out.
// ---------------------------------------------------------------------------
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseIters = 4;  // rows (2D) or planes (3D) per thread and level

template <int DIM>
struct CoarseMap {
    // thread -> (i, j, k) of iteration t; false when outside the level
    static __device__ __forceinline__ bool at(const Geo& g, int t, int& i, int& j, int& k) {
        const int tid = threadIdx.x;
        if (DIM == 2) {
            i = tid & 63;
            j = (tid >> 6) + 16 * t;
            k = 0;
        } else {
            i = tid & 15;
            j = (tid >> 4) & 15;
            k = (tid >> 8) + 4 * t;
        }
        return i < g.nx && j < g.ny && k < g.nz;
    }
};

__device__ __forceinline__ int cpad_idx(const Geo& g, int i, int j, int k) {
    const int px = g.nx + 4, py = g.ny + 4;
    return ((k + (g.dim == 3 ? 2 : 0)) * py + (j + 2)) * px + (i + 2);
}

template <typename T, int ORDER, int DIM>
__device__ __forceinline__ T lap_pad(const T* X, const Geo& g, int p, int i, int j, int k, T uc) {
    const int sy = g.nx + 4, sz = (g.nx + 4) * (g.ny + 4);
    T s = d2_lds<T, ORDER>(X, p, 1, i, g.nx, uc) * axis_coef<T, ORDER>(g.ihx2);
    s += d2_lds<T, ORDER>(X, p, sy, j, g.ny, uc) * axis_coef<T, ORDER>(g.ihy2);
    if (DIM == 3) s += d2_lds<T, ORDER>(X, p, sz, k, g.nz, uc) * axis_coef<T, ORDER>(g.ihz2);
    return s;
}

// Points of one colour: every lane owns one (2D: i = 2 (tid % 32) + parity,
// j = tid / 32 + 32 t; 3D: i = 2 (tid % 8) + parity, j = tid / 8 % 16,
// k = tid / 128 + 8 t), so two passes cover a 64 x 64 or 16^3 level.
constexpr int kCoarseColourIters = 2;
template <int DIM>
__device__ __forceinline__ bool colour_point(const Geo& g, int t, int colour, int& i, int& j, int& k) {
    const int tid = threadIdx.x;
    if (DIM == 2) {
        j = (tid >> 5) + 32 * t;
        k = 0;
        i = 2 * (tid & 31) + ((j + colour) & 1);
    } else {
        j = (tid >> 3) & 15;
        k = (tid >> 7) + 8 * t;
        i = 2 * (tid & 7) + ((j + k + colour) & 1);
    }
    return i < g.nx && j < g.ny && k < g.nz;
}

// Reciprocal of the diagonal of M at points whose stencil does not reach a ghost.
template <typename T, int ORDER, int DIM>
__device__ __forceinline__ T interior_inv_diag(const Geo& g, T a) {
    const T c0 = ORDER == 2 ? T(2) : T(30.0 / 12.0);
    T s = (T)g.ihx2 + (T)g.ihy2;
    if (DIM == 3) s += (T)g.ihz2;
    return T(1) / (T(1) + a * c0 * s);
}

template <typename T, int ORDER, int DIM>
__device__ void pad_half_sweep(T* x, const T* b, const Geo& g, T a, T w, int colour) {
    const T inv_diag = w * interior_inv_diag<T, ORDER, DIM>(g, a);
    T nv[kCoarseColourIters];
    int np[kCoarseColourIters];
#pragma unroll
    for (int t = 0; t < kCoarseColourIters; ++t) {
        np[t] = -1;
        int i, j, k;
        if (!colour_point<DIM>(g, t, colour, i, j, k)) continue;
        const int p = cpad_idx(g, i, j, k);
        const T xc = x[p];
        const T lap = lap_pad<T, ORDER, DIM>(x, g, p, i, j, k, xc);
        const T r = b[p] - (xc - a * lap);
        const bool edge = ORDER == 4 && (i == 0 || i == g.nx - 1 || j == 0 || j == g.ny - 1 ||
                                         (DIM == 3 && (k == 0 || k == g.nz - 1)));
        nv[t] = edge ? xc + (w * r) / mdiag_at<T, ORDER, DIM, false>(i, j, k, g, a) : xc + r * inv_diag;
        np[t] = p;
    }
    // Order 4 reads same-colour neighbours (old values) that other threads are
    // about to overwrite; order 2 reads only the other colour, and each point
    // of this colour only by the thread that updates it.
    if (ORDER == 4) __syncthreads();
#pragma unroll
    for (int t = 0; t < kCoarseColourIters; ++t)
        if (np[t] >= 0) x[np[t]] = nv[t];
    __syncthreads();
}

template <typename T, int DIM>
__device__ void pad_zero(T* x, const Geo& g) {
    const int tot = (g.nx + 4) * (g.ny + 4) * (DIM == 3 ? g.nz + 4 : 1);
    for (int q = threadIdx.x; q < tot; q += kCoarseThreads) x[q] = T(0);
}

// Residual b - M x of a level into the scratch array r (same padded layout),
// then full-weighting restriction of r into bc.
template <typename T, int ORDER, int DIM>
__device__ void pad_restrict(const T* x, const T* b, const Geo& gf, T a, T* bc, const Geo& gc, T* r) {
#pragma unroll
    for (int t = 0; t < kCoarseIters; ++t) {
        int i, j, k;
        if (!CoarseMap<DIM>::at(gf, t, i, j, k)) continue;
        const int p = cpad_idx(gf, i, j, k);
        const T xf = x[p];
        r[p] = b[p] - (xf - a * lap_pad<T, ORDER, DIM>(x, gf, p, i, j, k, xf));
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kCoarseIters; ++t) {
        int ic, jc, kc;
        if (!CoarseMap<DIM>::at(gc, t, ic, jc, kc)) continue;
        const int fi = 2 * ic + 1, fj = 2 * jc + 1, fk = (DIM == 3) ? 2 * kc + 1 : 0;
        T sum = T(0);
        const int zlo = (DIM == 3) ? -1 : 0, zhi = (DIM == 3) ? 1 : 0;
        for (int oz = zlo; oz <= zhi; ++oz) {
            T plane = T(0);
            for (int oy = -1; oy <= 1; ++oy) {
                T row = T(0);
                for (int ox = -1; ox <= 1; ++ox)
                    row += (ox == 0 ? T(0.5) : T(0.25)) * r[cpad_idx(gf, fi + ox, fj + oy, fk + oz)];
                plane += (oy == 0 ? T(0.5) : T(0.25)) * row;
            }
            sum += (DIM == 3) ? (oz == 0 ? T(0.5) : T(0.25)) * plane : plane;
        }
        bc[cpad_idx(gc, ic, jc, kc)] = sum;
    }
    __syncthreads();
}

// x_f += P x_c with the zero halo standing in for the walls.
template <typename T, int DIM>
__device__ void pad_prolong(T* xf, const Geo& gf, const T* xc, const Geo& gc) {
#pragma unroll
    for (int t = 0; t < kCoarseIters; ++t) {
        int i, j, k;
        if (!CoarseMap<DIM>::at(gf, t, i, j, k)) continue;
        int ci[2], cj[2], ck[2];
        T wi[2], wj[2], wk[2];
        ci[0] = (i - 1) >> 1; ci[1] = i >> 1; wi[0] = (i & 1) ? T(1) : T(0.5); wi[1] = (i & 1) ? T(0) : T(0.5);
        if (i & 1) ci[1] = ci[0];
        cj[0] = (j - 1) >> 1; cj[1] = j >> 1; wj[0] = (j & 1) ? T(1) : T(0.5); wj[1] = (j & 1) ? T(0) : T(0.5);
        if (j & 1) cj[1] = cj[0];
        if (DIM == 3) {
            ck[0] = (k - 1) >> 1; ck[1] = k >> 1; wk[0] = (k & 1) ? T(1) : T(0.5); wk[1] = (k & 1) ? T(0) : T(0.5);
            if (k & 1) ck[1] = ck[0];
        } else {
            ck[0] = ck[1] = 0; wk[0] = T(1); wk[1] = T(0);
        }
        T v = T(0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T plane = T(0);
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                T row = T(0);
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) row += wi[aa] * xc[cpad_idx(gc, ci[aa], cj[bb], ck[c])];
                plane += wj[bb] * row;
            }
            v += wk[c] * plane;
        }
        xf[cpad_idx(gf, i, j, k)] += v;
    }
    __syncthreads();
}

template <typename T, int ORDER, int DIM>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_vcycle(const T* __restrict__ b_in, const T* __restrict__ x_in,
                                                                  T* __restrict__ x_out, CoarseLevels c, T a, T w0,
                                                                  T w, int nu1, int nu2, int coarse_sweeps,
                                                                  T bscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* smem = reinterpret_cast<T*>(smem_raw);
    const int L = c.nlev;
    for (int l = 0; l < L; ++l) {
        pad_zero<T, DIM>(smem + c.off_x[l], c.g[l]);
        pad_zero<T, DIM>(smem + c.off_b[l], c.g[l]);
    }
    __syncthreads();
    {
        const Geo& g0 = c.g[0];
        T* x0 = smem + c.off_x[0];
        T* b0 = smem + c.off_b[0];
#pragma unroll
        for (int t = 0; t < kCoarseIters; ++t) {
            int i, j, k;
            if (!CoarseMap<DIM>::at(g0, t, i, j, k)) continue;
            const int64_t gq = lin(g0, i, j, k);
            const int p = cpad_idx(g0, i, j, k);
            b0[p] = bscale * b_in[gq];
            if (x_in) x0[p] = x_in[gq];
        }
        __syncthreads();
    }
    // weight of the kernel's first level w0 (the caller's level weight), w below
    for (int l = 0; l < L - 1; ++l) {
        T* x = smem + c.off_x[l];
        T* b = smem + c.off_b[l];
        const T wl = l == 0 ? w0 : w;
        for (int s = 0; s < nu1; ++s) {
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 0);
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 1);
        }
        pad_restrict<T, ORDER, DIM>(x, b, c.g[l], a, smem + c.off_b[l + 1], c.g[l + 1], smem + c.off_r);
    }
    {
        const int l = L - 1;
        T* x = smem + c.off_x[l];
        T* b = smem + c.off_b[l];
        // one point: a single half-sweep with weight 1 is the exact solve
        const bool one = c.g[l].size() == 1;
        const int sweeps = one ? 1 : coarse_sweeps;
        const T wl = one ? T(1) : (l == 0 ? w0 : w);
        for (int s = 0; s < sweeps; ++s) {
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 0);
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 1);
        }
    }
    for (int l = L - 2; l >= 0; --l) {
        T* x = smem + c.off_x[l];
        T* b = smem + c.off_b[l];
        pad_prolong<T, DIM>(x, c.g[l], smem + c.off_x[l + 1], c.g[l + 1]);
        const T wl = l == 0 ? w0 : w;
        for (int s = 0; s < nu2; ++s) {
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 0);
            pad_half_sweep<T, ORDER, DIM>(x, b, c.g[l], a, wl, 1);
        }
    }
    {
        const Geo& g0 = c.g[0];
        const T* x0 = smem + c.off_x[0];
#pragma unroll
        for (int t = 0; t < kCoarseIters; ++t) {
            int i, j, k;
            if (!CoarseMap<DIM>::at(g0, t, i, j, k)) continue;
            x_out[lin(g0, i, j, k)] = x0[cpad_idx(g0, i, j, k)];
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T, int ORDER, int DIM, int TX, int TY, int TZ>
static hipError_t sweep_dispatch_tile(const T* xin, const T* xc, const T* b, T bs, T* xout, const Geo& g,
                                      const Geo& gc, T a, T w, bool zero_in, bool prolong, hipStream_t s) {
    dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, DIM == 3 ? (g.nz + TZ - 1) / TZ : 1);
#define EW_ST(Z, P)                                                                                              \
    do {                                                                                                         \
        if (g.wall)                                                                                              \
            k_sweep_tile<T, ORDER, DIM, Z, P, true, TX, TY, TZ><<<grid, kTileThreads, 0, s>>>(xin, xc, b, bs, xout, g, gc, a, w); \
        else                                                                                                     \
            k_sweep_tile<T, ORDER, DIM, Z, P, false, TX, TY, TZ><<<grid, kTileThreads, 0, s>>>(xin, xc, b, bs, xout, g, gc, a, w); \
    } while (0)
    if (zero_in && prolong) EW_ST(true, true);
    else if (zero_in) EW_ST(true, false);
    else if (prolong) EW_ST(false, true);
    else EW_ST(false, false);
#undef EW_ST
    return hipGetLastError();
}

// 32 x 8 x 8 tiles from 1024 of them up (127^3 and larger); 16 x 8 x 4 tiles
// (less serial work per workgroup, 8 times as many workgroups) on smaller
// levels, where the large tiles leave most CUs idle.
// Order-2 3D levels without walls march 64 x 8 column tiles through chunks
// of 16 planes (8 where 16 give fewer than 1024 workgroups) when chunks of 8
// give at least 512 workgroups.  On 255^3 (FP32) chunks of 16 (2048
// workgroups) measured faster than chunks sized so that every workgroup is
// resident at once (22 planes, 1536) and than chunks of 11 (3072).
template <typename T>
static bool sweep_z3d_dispatch(const T* xin, const T* xc, const T* b, T bs, T* xout, const Geo& g, const Geo& gc,
                               double a, double w, bool zero_in, bool prolong, hipStream_t s, hipError_t* err) {
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    if (cols * ((g.nz + 7) / 8) < 512) return false;
    if (prolong && zero_in) return false;  // not a V-cycle combination
    const T inv = (T)(w / (1.0 + 2.0 * a * (g.ihx2 + g.ihy2 + g.ihz2)));
    const T aa = (T)a;
    const int cz = cols * ((g.nz + 15) / 16) >= 1024 ? 16 : 8;
    dim3 grid((g.nx + 63) / 64, (g.ny + 7) / 8, (g.nz + cz - 1) / cz);
#define EW_Z3D(Z, P) k_sweep_z3d<T, Z, P, 8><<<grid, kTileThreads, 0, s>>>(xin, xc, b, bs, xout, g, gc, aa, inv, cz)
    if (prolong) EW_Z3D(false, true);
    else if (zero_in) EW_Z3D(true, false);
    else EW_Z3D(false, false);
#undef EW_Z3D
    *err = hipGetLastError();
    return true;
}

bool sweep_z3d_fuses_prolong(const Geo& g, int order) {
    if (g.dim != 3 || order != 2 || g.wall) return false;
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    return cols * ((g.nz + 7) / 8) >= 512;
}

template <typename T, int ORDER, int DIM>
static hipError_t sweep_dispatch(const T* xin, const T* xc, const T* b, T bs, T* xout, const Geo& g, const Geo& gc,
                                 T a, T w, bool zero_in, bool prolong, hipStream_t s) {
    constexpr int TX = SweepTile<DIM>::TX, TY = SweepTile<DIM>::TY, TZ = SweepTile<DIM>::TZ;
    const int64_t big = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
    if (DIM == 3 && big < 1024)
        return sweep_dispatch_tile<T, ORDER, DIM, 16, 8, 4>(xin, xc, b, bs, xout, g, gc, a, w, zero_in, prolong, s);
    return sweep_dispatch_tile<T, ORDER, DIM, TX, TY, TZ>(xin, xc, b, bs, xout, g, gc, a, w, zero_in, prolong, s);
}

template <typename T>
hipError_t launch_sweep_tile(const T* xin, const T* xc, const T* b, double bscale, T* xout, const Geo& g,
                             const Geo& gc, int order, double a, double w, bool zero_in, bool prolong,
                             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const T bs = (T)bscale, aa = (T)a, ww = (T)w;
    if (g.dim == 2)
        return launch_sweep2d<T>(xin, xc, b, bscale, xout, g, gc, order, a, w, zero_in, prolong, s, ev0, ev1);
    if (ev0) EW_RET_ON_ERR(hipEventRecord(ev0, s));
    hipError_t e = hipSuccess;
    if (!(order == 2 && !g.wall && sweep_z3d_dispatch<T>(xin, xc, b, bs, xout, g, gc, a, w, zero_in, prolong, s, &e)))
        e = order == 2 ? sweep_dispatch<T, 2, 3>(xin, xc, b, bs, xout, g, gc, aa, ww, zero_in, prolong, s)
                       : sweep_dispatch<T, 4, 3>(xin, xc, b, bs, xout, g, gc, aa, ww, zero_in, prolong, s);
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    return e;
}

template <typename T, int ORDER, int DIM>
static hipError_t restrict_dispatch(const T* x, const T* b, T bs, const Geo& gf, T a, T* bc, const Geo& gc,
                                    hipStream_t s) {
    constexpr int CX = RestrictTile<DIM>::CX, CY = RestrictTile<DIM>::CY, CZ = RestrictTile<DIM>::CZ;
    constexpr int NT = RestrictTile<DIM>::NT;
    // short tiles (less serial work per block) below 512 tall ones (coarse
    // grids smaller than 511^2; measured on the 1023^2 level in XCD order)
    const int64_t tall = (int64_t)((gc.nx + CX - 1) / CX) * ((gc.ny + CY - 1) / CY) * (DIM == 3 ? (gc.nz + CZ - 1) / CZ : 1);
    if (DIM == 2 && tall < 512) {
        dim3 grid((gc.nx + CX - 1) / CX, (gc.ny + 3) / 4, 1);
        if (gf.wall) k_restrict_tile<T, ORDER, DIM, 4, true, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
        else k_restrict_tile<T, ORDER, DIM, 4, false, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
    } else if (DIM == 2) {
        // 32 x 8 coarse tiles: half the LDS of 32 x 16, twice the workgroups per CU
        dim3 grid((gc.nx + CX - 1) / CX, (gc.ny + 7) / 8, 1);
        if (gf.wall) k_restrict_tile<T, ORDER, DIM, 8, true, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
        else k_restrict_tile<T, ORDER, DIM, 8, false, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
    } else {
        dim3 grid((gc.nx + CX - 1) / CX, (gc.ny + CY - 1) / CY, DIM == 3 ? (gc.nz + CZ - 1) / CZ : 1);
        if (gf.wall) k_restrict_tile<T, ORDER, DIM, CY, true, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
        else k_restrict_tile<T, ORDER, DIM, CY, false, NT><<<grid, NT, 0, s>>>(x, b, bs, gf, a, bc, gc);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_tile(const T* x, const T* b, double bscale, const Geo& gf, int order, double a, T* bc,
                                const Geo& gc, hipStream_t s) {
    const T bs = (T)bscale, aa = (T)a;
    if (gf.dim == 2) {
        if (order == 2) return restrict_dispatch<T, 2, 2>(x, b, bs, gf, aa, bc, gc, s);
        return restrict_dispatch<T, 4, 2>(x, b, bs, gf, aa, bc, gc, s);
    }
    if (order == 2) return restrict_dispatch<T, 2, 3>(x, b, bs, gf, aa, bc, gc, s);
    return restrict_dispatch<T, 4, 3>(x, b, bs, gf, aa, bc, gc, s);
}

template <typename T>
hipError_t launch_coarse_vcycle(const T* b, double bscale, const T* x_in, T* x_out, const CoarseLevels& c, int order,
                                double a, double w0, double w, int nu1, int nu2, int coarse_sweeps, hipStream_t s) {
    const size_t lds = (size_t)c.lds_elems * sizeof(T);
    const T aa = (T)a, bs = (T)bscale, ww0 = (T)w0, ww = (T)w;
    if (c.g[0].dim == 2) {
        if (order == 2) k_coarse_vcycle<T, 2, 2><<<1, kCoarseThreads, lds, s>>>(b, x_in, x_out, c, aa, ww0, ww, nu1, nu2, coarse_sweeps, bs);
        else k_coarse_vcycle<T, 4, 2><<<1, kCoarseThreads, lds, s>>>(b, x_in, x_out, c, aa, ww0, ww, nu1, nu2, coarse_sweeps, bs);
    } else {
        if (order == 2) k_coarse_vcycle<T, 2, 3><<<1, kCoarseThreads, lds, s>>>(b, x_in, x_out, c, aa, ww0, ww, nu1, nu2, coarse_sweeps, bs);
        else k_coarse_vcycle<T, 4, 3><<<1, kCoarseThreads, lds, s>>>(b, x_in, x_out, c, aa, ww0, ww, nu1, nu2, coarse_sweeps, bs);
    }
    return hipGetLastError();
}

// Dynamic LDS above 64 KB must be enabled per kernel.
template <typename T>
hipError_t prepare_coarse_vcycle(int dim, int order, size_t lds_bytes) {
    const void* f = nullptr;
    if (dim == 2) f = order == 2 ? (const void*)k_coarse_vcycle<T, 2, 2> : (const void*)k_coarse_vcycle<T, 4, 2>;
    else f = order == 2 ? (const void*)k_coarse_vcycle<T, 2, 3> : (const void*)k_coarse_vcycle<T, 4, 3>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

#define EW_INST_TILE(T)                                                                                          \
    template hipError_t launch_sweep_tile<T>(const T*, const T*, const T*, double, T*, const Geo&, const Geo&,    \
                                             int, double, double, bool, bool, hipStream_t, hipEvent_t,            \
                                             hipEvent_t);                                                         \
    template hipError_t launch_restrict_tile<T>(const T*, const T*, double, const Geo&, int, double, T*,         \
                                                const Geo&, hipStream_t);                                         \
    template hipError_t launch_coarse_vcycle<T>(const T*, double, const T*, T*, const CoarseLevels&, int, double, double, \
                                                double, int, int, int, hipStream_t);                              \
    template hipError_t prepare_coarse_vcycle<T>(int, int, size_t);
EW_INST_TILE(double)
EW_INST_TILE(float)
#undef EW_INST_TILE

}  // namespace ew
