// The finest-level smoother for 2D grids: one full red-black Gauss-Seidel
// sweep of M = I - a L_h per pass over memory, tiled through LDS (the kernel
// that dominates the implicit wave-solve on large 2D grids).
#include <hip/hip_ext.h>

#include <type_traits>

#include "mg_tile.h"
#include "stencil_dev.h"

namespace ew {

// Threads per workgroup (same-box A/B measurements, rocprofv3 averages):
//  * the fused two-sweep pass: 512, i.e. 32 wavefronts per CU instead of 20
//    (four workgroups fit the LDS either way): 1 % faster on 2047^2, 4 % on
//    1023^2 than 256;
//  * the single sweep: 256 on 64 x 16 tiles (512 measured 2 % slower on
//    2047^2), 512 on the 64 x 8 tiles of small levels (255^2: 5.6 -> 4.4 us);
//  * the fused two-sweep + restriction pass of small levels, where the time
//    per tile, not the bytes, sets the pace: 1024 (255^2: 8.3 us with 256,
//    6.2 with 512, 5.6 with 1024).
constexpr int kSweep2xThreads = 512;
template <int TY>
constexpr int single_sweep_threads() {
    return TY >= 16 ? 256 : 512;
}
constexpr int kSweep2xRestrictThreads = 1024;

// ---------------------------------------------------------------------------
// 2D sweep, one tile of 64 x TY outputs per workgroup.  x is staged in LDS
// with a halo of H = R + 1, b with a halo of 1; with PROLONG the coarse
// values under the tile are staged as well and interpolated from LDS.  During
// each half-sweep every lane owns one point of the colour being relaxed, so
// no lane idles on a point of the other colour.  Interior points multiply by
// the reciprocal of the constant interior diagonal; points whose diagonal
// carries an order-4 ghost divide.
// ---------------------------------------------------------------------------
// The relaxation phases of NS = 1 or 2 red-black sweeps of one 64 x TY tile
// by NT threads, after staging: x in X with a halo of R + 2 NS - 1, b in B
// with a halo of 2 NS - 1.  Each half-sweep but the last relaxes the tile
// plus one layer more than the next one needs; the last (black) half-sweep
// is written out with the red points beside it.  NW selects the Neumann-wall
// closures; IN drops the tests a tile inside the grid does not need.
template <typename T, int ORDER, int TY, bool NW, bool IN, int NS, int NT>
__device__ __forceinline__ void sweep_phases(T* X, const T* B, int tid, int x0, int y0, const Geo& g, T a,
                                             T inv_diag, T w, T* __restrict__ xout) {
    static_assert(NS == 1 || NS == 2, "one or two sweeps per pass");
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, H = R + 2 * NS - 1;
    constexpr int LX = TX + 2 * H;
    constexpr int BH = 2 * NS - 1, BX = TX + 2 * BH;
    static_assert(LX % 2 == 0 && BX % 2 == 0 && TY % 2 == 0, "row pairs of opposite column parities");
    const T cxc = axis_coef<T, ORDER>(g.ihx2), cyc = axis_coef<T, ORDER>(g.ihy2);
    // relaxed value of global point (gi, gj) from the values now in LDS
    auto relax = [&](int gi, int gj) -> T {
        const int p = (gj - y0 + H) * LX + (gi - x0 + H);
        const T bval = B[(gj - y0 + BH) * BX + (gi - x0 + BH)];
        const T uc = X[p];
        T dx, dy;
        if (NW) {
            dx = d2_framed<T, ORDER>(X, p, 1, gi, g.nx, uc, g.wall & 3);
            dy = d2_framed<T, ORDER>(X, p, LX, gj, g.ny, uc, (g.wall >> 2) & 3);
        } else if (ORDER == 2) {
            dx = X[p - 1] + X[p + 1] - T(2) * uc;
            dy = X[p - LX] + X[p + LX] - T(2) * uc;
        } else {
            const T l2 = (!IN && gi == 0) ? -uc : X[p - 2];
            const T r2 = (!IN && gi == g.nx - 1) ? -uc : X[p + 2];
            const T d2 = (!IN && gj == 0) ? -uc : X[p - 2 * LX];
            const T u2 = (!IN && gj == g.ny - 1) ? -uc : X[p + 2 * LX];
            dx = T(16) * (X[p - 1] + X[p + 1]) - (l2 + r2) - T(30) * uc;
            dy = T(16) * (X[p - LX] + X[p + LX]) - (d2 + u2) - T(30) * uc;
        }
        const T r = bval - (uc - a * (dx * cxc + dy * cyc));
        const bool edge = !IN && ORDER == 4 && (NW ? (gi <= 1 || gi >= g.nx - 2 || gj <= 1 || gj >= g.ny - 2)
                                            : (gi == 0 || gi == g.nx - 1 || gj == 0 || gj == g.ny - 1));
        return edge ? uc + (w * r) / mdiag_w<T, ORDER, 2>(gi, gj, 0, g, a, NW ? g.wall : 0) : uc + r * inv_diag;
    };
    // one half-sweep of colour `colour` on the tile plus K layers: new values to
    // registers (same-colour neighbours must be read old), then into LDS
    auto half = [&](auto kc, int colour) {
        constexpr int K = decltype(kc)::value;
        constexpr int W2 = (TX + 2 * K) / 2, NR = TY + 2 * K, NP = NR * W2;
        constexpr int IT = (NP + NT - 1) / NT;
        T rv[IT];
        int rp[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            rp[t] = -1;
            const int idx = tid + t * NT;
            if (idx >= NP) continue;
            // lanes alternate between the two rows of a pair, whose points of
            // one colour sit in columns of opposite parity (LX and BX are
            // even), so consecutive lanes read distinct LDS banks (the row
            // count is even)
            const int pr = idx / (2 * W2), q2 = idx - pr * (2 * W2);
            const int r = 2 * pr + (q2 & 1), k2 = q2 >> 1;
            const int gj = y0 - K + r;
            const int gi = x0 - K + ((colour + gj + x0 - K) & 1) + 2 * k2;
            if (!IN && (gj < 0 || gj >= g.ny || gi < 0 || gi >= g.nx)) continue;
            rv[t] = relax(gi, gj);
            rp[t] = (gj - y0 + H) * LX + (gi - x0 + H);
        }
        if (ORDER == 4) __syncthreads();  // same-colour neighbours are read old (order 4 only)
#pragma unroll
        for (int t = 0; t < IT; ++t)
            if (rp[t] >= 0) X[rp[t]] = rv[t];
        __syncthreads();
    };
    if constexpr (NS == 2) {
        half(std::integral_constant<int, 3>{}, 0);  // red, first sweep
        half(std::integral_constant<int, 2>{}, 1);  // black, first sweep
    }
    half(std::integral_constant<int, 1>{}, 0);  // red, last sweep
    // black of the last sweep on the tile, written out with the red point of
    // the same pair of columns
    constexpr int NP = TY * (TX / 2), IT = (NP + NT - 1) / NT;
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int idx = tid + t * NT;
        if (idx >= NP) continue;
        const int pr = idx / TX, q2 = idx - pr * TX;  // row pairs, as in `half`
        const int r = 2 * pr + (q2 & 1), k2 = q2 >> 1;
        const int gj = y0 + r;
        const int gib = x0 + ((1 + gj) & 1) + 2 * k2, gir = gib ^ 1;
        if (!IN && gj >= g.ny) continue;
        T* row = xout + (int64_t)gj * g.nx;
        if (IN || gib < g.nx) row[gib] = relax(gib, gj);
        if (IN || gir < g.nx) row[gir] = X[(gj - y0 + H) * LX + (gir - x0 + H)];
    }
}

// Staging and phases of k_sweep_tile2d for one tile; IN: the tile lies
// inside the grid with its halo (tile_inside2d), so no load or relaxed point
// needs a bounds, ghost or wall test.
template <typename T, int ORDER, int TY, bool ZERO_IN, bool PROLONG, bool WALLS, bool IN, int NT>
__device__ __forceinline__ void sweep_tile2d_body(const T* __restrict__ xin, const T* __restrict__ xc,
                                                  const T* __restrict__ b, T bscale, T* __restrict__ xout,
                                                  const Geo& g, const Geo& gc, T a, T inv_diag, T w, T* X, T* B,
                                                  T* XC, int tid, int x0, int y0, bool nw) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, H = R + 1;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BX = TX + 2, BY = TY + 2;
    constexpr int CXW = (LX + 5) / 2 + 1, CYW = (LY + 5) / 2 + 1;  // coarse cells under the x tile
    const int cx0 = PROLONG ? (x0 - H - 1) >> 1 : 0, cy0 = PROLONG ? (y0 - H - 1) >> 1 : 0;

    // Staging: every global load of a thread is issued (into registers) before
    // its first LDS store, so a block waits for memory once, not once per row.
    constexpr int NX = LY * LX, NB = BY * BX, NC = PROLONG ? CYW * CXW : 0;
    constexpr int IX = (NX + NT - 1) / NT;
    constexpr int IB = (NB + NT - 1) / NT;
    constexpr int IC = PROLONG ? (NC + NT - 1) / NT : 1;
    T cv[IC], xv[IX], bv[IB];
#pragma unroll
    for (int t = 0; t < IC; ++t) {
        const int q = tid + t * NT;
        T v = T(0);
        if (PROLONG && q < NC) {
            const int cy = q / CXW, cxx = q - cy * CXW;
            const int ic = cx0 + cxx, jc = cy0 + cy;
            if (ic >= 0 && ic < gc.nx && jc >= 0 && jc < gc.ny) v = xc[(int64_t)jc * gc.nx + ic];
        }
        cv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * NT;
        T v = T(0);
        if (!ZERO_IN && q < NX) {
            const int ly = q / LX, lx = q - ly * LX;
            const int gi = x0 - H + lx, gj = y0 - H + ly;
            if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = xin[(int64_t)gj * g.nx + gi];
        }
        xv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * NT;
        T v = T(0);
        if (q < NB) {
            const int by = q / BX, bx = q - by * BX;
            const int gi = x0 - 1 + bx, gj = y0 - 1 + by;
            if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = b[(int64_t)gj * g.nx + gi];
        }
        bv[t] = v;  // scaled at the LDS store: no arithmetic on a load in flight
    }
    if (PROLONG) {
#pragma unroll
        for (int t = 0; t < IC; ++t) {
            const int q = tid + t * NT;
            if (q < NC) XC[q] = cv[t];
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * NT;
        if (q < NX) {
            T v = xv[t];
            if (PROLONG) {
                const int ly = q / LX, lx = q - ly * LX;
                const int gi = x0 - H + lx, gj = y0 - H + ly;
                if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) {
                    // q = f - off (off = 1 behind a Dirichlet low wall, 0 behind a
                    // Neumann one): q even -> coarse q/2; odd -> mean of (q-1)/2 and (q+1)/2
                    const int qi = WALLS ? gi - ((g.wall & 1) ? 0 : 1) : gi - 1;
                    const int qj = WALLS ? gj - ((g.wall & 4) ? 0 : 1) : gj - 1;
                    const int ia = (qi >> 1) - cx0, ib = ((qi + 1) >> 1) - cx0;
                    const int ja = (qj >> 1) - cy0, jb = ((qj + 1) >> 1) - cy0;
                    const T wia = (qi & 1) ? T(0.5) : T(1), wib = (qi & 1) ? T(0.5) : T(0);
                    const T wja = (qj & 1) ? T(0.5) : T(1), wjb = (qj & 1) ? T(0.5) : T(0);
                    const T rowa = wia * XC[ja * CXW + ia] + wib * XC[ja * CXW + ib];
                    const T rowb = wia * XC[jb * CXW + ia] + wib * XC[jb * CXW + ib];
                    v += wja * rowa + wjb * rowb;
                }
            }
            X[q] = v;
        }
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * NT;
        if (q < NB) B[q] = bscale * bv[t];
    }
    __syncthreads();

    // tiles near a Neumann wall run the wall closures; all others the
    // Dirichlet-only code (a uniform branch, taken once per tile)
    if constexpr (IN) {
        sweep_phases<T, ORDER, TY, false, true, 1, NT>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    } else if constexpr (WALLS) {
        if (nw) sweep_phases<T, ORDER, TY, true, false, 1, NT>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
        else sweep_phases<T, ORDER, TY, false, false, 1, NT>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    } else {
        sweep_phases<T, ORDER, TY, false, false, 1, NT>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    }
}

template <typename T, int ORDER, int TY, bool ZERO_IN, bool PROLONG, bool WALLS>
__global__ __launch_bounds__(single_sweep_threads<TY>()) void k_sweep_tile2d(
    const T* __restrict__ xin, const T* __restrict__ xc, const T* __restrict__ b, T bscale, T* __restrict__ xout,
    Geo g, Geo gc, T a, T inv_diag, T w) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, H = R + 1;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BX = TX + 2, BY = TY + 2;
    constexpr int CXW = (LX + 5) / 2 + 1, CYW = (LY + 5) / 2 + 1;
    __shared__ T X[LY * LX];
    __shared__ T B[BY * BX];
    __shared__ T XC[PROLONG ? CYW * CXW : 1];
    const int tid = threadIdx.x;
    int bx, by;
    xcd_block(bx, by);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY;
    const bool nw = WALLS && near_neumann(g, x0, x0 + TX, y0, y0 + TY, 0, 1, H);  // uniform per tile
    if (!nw && tile_inside2d(g, x0, x0 + TX, y0, y0 + TY, H))
        sweep_tile2d_body<T, ORDER, TY, ZERO_IN, PROLONG, WALLS, true, single_sweep_threads<TY>()>(
            xin, xc, b, bscale, xout, g, gc, a, inv_diag, w, X, B, XC, tid, x0, y0, nw);
    else
        sweep_tile2d_body<T, ORDER, TY, ZERO_IN, PROLONG, WALLS, false, single_sweep_threads<TY>()>(
            xin, xc, b, bscale, xout, g, gc, a, inv_diag, w, X, B, XC, tid, x0, y0, nw);
}

// ---------------------------------------------------------------------------
// Two consecutive red-black sweeps of one 64 x TY tile from one staging of x
// and b: red on the tile plus 3 layers, black on plus 2, red on plus 1, black
// on the tile (each half-sweep relaxes one colour from the values before it,
// so every phase needs the previous one on a region one layer wider, and the
// order-4 same-colour neighbours two layers wider).  x is staged with a halo
// of R + 3, b with a halo of 3.  The result equals two calls of the single
// sweep bit for bit: every relaxed value is computed by the same expression
// from the same inputs.  Halves the HBM traffic of the two pre-smoothing
// sweeps and saves one launch per level.  (A layout with one LDS array per
// colour, which makes the lanes' LDS reads contiguous, measured slower.)
// ---------------------------------------------------------------------------
// Staging and phases of k_sweep2x_tile2d for one tile; IN as in
// sweep_tile2d_body.
template <typename T, int ORDER, int TY, bool ZERO_IN, bool WALLS, bool IN>
__device__ __forceinline__ void sweep2x_body(const T* __restrict__ xin, const T* __restrict__ b, T bscale,
                                             T* __restrict__ xout, const Geo& g, T a, T inv_diag, T w, T* X, T* B,
                                             int tid, int x0, int y0, bool nw) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, H = R + 3;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BH = 3, BX = TX + 2 * BH, BY = TY + 2 * BH;

    // staging, every global load issued before the first LDS store
    constexpr int NX = LY * LX, NB = BY * BX;
    constexpr int IX = (NX + kSweep2xThreads - 1) / kSweep2xThreads;
    constexpr int IB = (NB + kSweep2xThreads - 1) / kSweep2xThreads;
    T xv[IX], bv[IB];
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kSweep2xThreads;
        T v = T(0);
        if (!ZERO_IN && q < NX) {
            const int ly = q / LX, lx = q - ly * LX;
            const int gi = x0 - H + lx, gj = y0 - H + ly;
            if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = xin[(int64_t)gj * g.nx + gi];
        }
        xv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * kSweep2xThreads;
        T v = T(0);
        if (q < NB) {
            const int by = q / BX, bx = q - by * BX;
            const int gi = x0 - BH + bx, gj = y0 - BH + by;
            if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = b[(int64_t)gj * g.nx + gi];
        }
        bv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < IX; ++t) {
        const int q = tid + t * kSweep2xThreads;
        if (q < NX) X[q] = xv[t];
    }
#pragma unroll
    for (int t = 0; t < IB; ++t) {
        const int q = tid + t * kSweep2xThreads;
        if (q < NB) B[q] = bscale * bv[t];
    }
    __syncthreads();

    if constexpr (IN) {
        sweep_phases<T, ORDER, TY, false, true, 2, kSweep2xThreads>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    } else if constexpr (WALLS) {
        if (nw)
            sweep_phases<T, ORDER, TY, true, false, 2, kSweep2xThreads>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
        else
            sweep_phases<T, ORDER, TY, false, false, 2, kSweep2xThreads>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    } else {
        sweep_phases<T, ORDER, TY, false, false, 2, kSweep2xThreads>(X, B, tid, x0, y0, g, a, inv_diag, w, xout);
    }
}

template <typename T, int ORDER, int TY, bool ZERO_IN, bool WALLS>
__global__ __launch_bounds__(kSweep2xThreads) void k_sweep2x_tile2d(const T* __restrict__ xin, const T* __restrict__ b,
                                                                 T bscale, T* __restrict__ xout, Geo g, T a,
                                                                 T inv_diag, T w) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, H = R + 3;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BH = 3, BX = TX + 2 * BH, BY = TY + 2 * BH;
    __shared__ T X[LY * LX];
    __shared__ T B[BY * BX];
    const int tid = threadIdx.x;
    int bx, by;
    xcd_block(bx, by);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY;
    const bool nw = WALLS && near_neumann(g, x0, x0 + TX, y0, y0 + TY, 0, 1, H);  // uniform per tile
    if (!nw && tile_inside2d(g, x0, x0 + TX, y0, y0 + TY, H))
        sweep2x_body<T, ORDER, TY, ZERO_IN, WALLS, true>(xin, b, bscale, xout, g, a, inv_diag, w, X, B, tid, x0, y0,
                                                         nw);
    else
        sweep2x_body<T, ORDER, TY, ZERO_IN, WALLS, false>(xin, b, bscale, xout, g, a, inv_diag, w, X, B, tid, x0, y0,
                                                          nw);
}

// hipExtLaunchKernelGGL records ev0/ev1 (when given) at the dispatch's own
// start and end, so profiling this kernel adds no separate event commands.
template <typename T, int ORDER, int TY, bool WALLS>
static hipError_t sweep2d_launch(const T* xin, const T* xc, const T* b, T bs, T* xout, const Geo& g, const Geo& gc,
                                 T aa, T inv, T w, bool zero_in, bool prolong, hipStream_t s, hipEvent_t ev0,
                                 hipEvent_t ev1) {
    dim3 grid((g.nx + 63) / 64, (g.ny + TY - 1) / TY, 1);
    dim3 block(single_sweep_threads<TY>());
    if (zero_in && prolong)
        hipExtLaunchKernelGGL((k_sweep_tile2d<T, ORDER, TY, true, true, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, xc, b, bs, xout, g, gc, aa, inv, w);
    else if (zero_in)
        hipExtLaunchKernelGGL((k_sweep_tile2d<T, ORDER, TY, true, false, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, xc, b, bs, xout, g, gc, aa, inv, w);
    else if (prolong)
        hipExtLaunchKernelGGL((k_sweep_tile2d<T, ORDER, TY, false, true, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, xc, b, bs, xout, g, gc, aa, inv, w);
    else
        hipExtLaunchKernelGGL((k_sweep_tile2d<T, ORDER, TY, false, false, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, xc, b, bs, xout, g, gc, aa, inv, w);
    return hipGetLastError();
}

template <typename T, int ORDER>
static hipError_t sweep2d_dispatch(const T* xin, const T* xc, const T* b, T bs, T* xout, const Geo& g, const Geo& gc,
                                   double a, double w, bool zero_in, bool prolong, hipStream_t s, hipEvent_t ev0,
                                   hipEvent_t ev1) {
    // interior diagonal of M = I - a L: 1 + a c_0 (1/hx^2 + 1/hy^2), c_0 = 2 (order 2) or 30/12 (order 4);
    // the relaxation weight w is folded into its reciprocal
    const double c0 = ORDER == 2 ? 2.0 : 30.0 / 12.0;
    const T inv = (T)(w / (1.0 + a * c0 * (g.ihx2 + g.ihy2)));
    const T ww = (T)w;
    const T aa = (T)a;
    // 64 x 16 tiles (22 KB of LDS, 7 workgroups per CU) from 1024 tiles up
    // (1023^2 and larger), 64 x 8 (less serial work per block) on smaller
    // levels; measured faster than 64 x 32 tiles on 2047^2, and on 1023^2
    // than 64 x 8 once the tiles run in XCD order
    const int64_t tiles16 = (int64_t)((g.nx + 63) / 64) * ((g.ny + 15) / 16);
    if (g.wall) {
        if (tiles16 >= 1024)
            return sweep2d_launch<T, ORDER, 16, true>(xin, xc, b, bs, xout, g, gc, aa, inv, ww, zero_in, prolong, s, ev0, ev1);
        return sweep2d_launch<T, ORDER, 8, true>(xin, xc, b, bs, xout, g, gc, aa, inv, ww, zero_in, prolong, s, ev0, ev1);
    }
    if (tiles16 >= 1024)
        return sweep2d_launch<T, ORDER, 16, false>(xin, xc, b, bs, xout, g, gc, aa, inv, ww, zero_in, prolong, s, ev0, ev1);
    return sweep2d_launch<T, ORDER, 8, false>(xin, xc, b, bs, xout, g, gc, aa, inv, ww, zero_in, prolong, s, ev0, ev1);
}

template <typename T, int ORDER, int TY, bool WALLS>
static hipError_t sweep2x_launch(const T* xin, const T* b, T bs, T* xout, const Geo& g, T aa, T inv, T w,
                                 bool zero_in, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    dim3 grid((g.nx + 63) / 64, (g.ny + TY - 1) / TY, 1);
    dim3 block(kSweep2xThreads);
    if (zero_in)
        hipExtLaunchKernelGGL((k_sweep2x_tile2d<T, ORDER, TY, true, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, b, bs, xout, g, aa, inv, w);
    else
        hipExtLaunchKernelGGL((k_sweep2x_tile2d<T, ORDER, TY, false, WALLS>), grid, block, 0, s, ev0, ev1, 0, xin, b, bs, xout, g, aa, inv, w);
    return hipGetLastError();
}

template <typename T, int ORDER>
static hipError_t sweep2x_dispatch(const T* xin, const T* b, T bs, T* xout, const Geo& g, double a, double w,
                                   bool zero_in, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const double c0 = ORDER == 2 ? 2.0 : 30.0 / 12.0;
    const T inv = (T)(w / (1.0 + a * c0 * (g.ihx2 + g.ihy2)));
    const T ww = (T)w;
    const T aa = (T)a;
    const int64_t tiles16 = (int64_t)((g.nx + 63) / 64) * ((g.ny + 15) / 16);
    if (g.wall) {
        if (tiles16 >= 1024) return sweep2x_launch<T, ORDER, 16, true>(xin, b, bs, xout, g, aa, inv, ww, zero_in, s, ev0, ev1);
        return sweep2x_launch<T, ORDER, 8, true>(xin, b, bs, xout, g, aa, inv, ww, zero_in, s, ev0, ev1);
    }
    if (tiles16 >= 1024) return sweep2x_launch<T, ORDER, 16, false>(xin, b, bs, xout, g, aa, inv, ww, zero_in, s, ev0, ev1);
    return sweep2x_launch<T, ORDER, 8, false>(xin, b, bs, xout, g, aa, inv, ww, zero_in, s, ev0, ev1);
}

template <typename T>
hipError_t launch_sweep2x2d(const T* xin, const T* b, double bscale, T* xout, const Geo& g, int order, double a,
                            double w, bool zero_in, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const T bs = (T)bscale;
    if (order == 2) return sweep2x_dispatch<T, 2>(xin, b, bs, xout, g, a, w, zero_in, s, ev0, ev1);
    return sweep2x_dispatch<T, 4>(xin, b, bs, xout, g, a, w, zero_in, s, ev0, ev1);
}

template hipError_t launch_sweep2x2d<double>(const double*, const double*, double, double*, const Geo&, int, double,
                                             double, bool, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sweep2x2d<float>(const float*, const float*, double, float*, const Geo&, int, double,
                                            double, bool, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------------------
// The two pre-smoothing sweeps of k_sweep2x_tile2d followed, from the same
// staging, by the residual r = bscale b - M x of the result and its
// full-weighting restriction (the work of k_restrict_tile), for 2D levels
// without Neumann walls.  The coarse points of a 64 x TY tile are the 32 x
// TY/2 whose fine centres 2I + 1, 2J + 1 lie in it; their weights reach one
// fine row and column beyond the tile, where r needs x one stencil radius
// further.  So the four half-sweeps relax the tile plus M + 3, M + 2, M + 1
// and M layers (M = R + 1), x is staged with a halo of R + M + 3 and b with
// M + 3, every half-sweep writes to LDS, and the tile is written out after
// the last.  r is formed with the same expressions as k_restrict_tile, over
// the (64 + 1) x (TY + 1) fine points from the tile's corner, into the LDS of
// b (no longer needed), and restricted from there.
// ---------------------------------------------------------------------------
// One tile of k_sweep2x_restrict_tile2d; IN: the tile lies inside the grid
// with its staged halo (tile_inside2d), so no load, relaxed point or residual
// point needs a bounds, ghost or wall-diagonal test.
template <typename T, int ORDER, int TY, bool ZERO_IN, bool IN>
__device__ __forceinline__ void sweep2x_restrict_body(const T* __restrict__ xin, const T* __restrict__ b, T bscale,
                                                      T* __restrict__ xout, const Geo& g, T a, T inv_diag, T w,
                                                      T* __restrict__ bc, const Geo& gc, T* X, T* B, int tid, int x0,
                                                      int y0) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, M = R + 1, H = R + M + 3;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BH = M + 3, BX = TX + 2 * BH, BY = TY + 2 * BH;
    constexpr int RX = TX + 1, RY = TY + 1, NR = RX * RY;
    static_assert(NR <= BX * BY, "the residual reuses the LDS of b");
    static_assert(TY % 2 == 0, "coarse rows pair fine rows");
    static_assert(LX % 2 == 0 && BX % 2 == 0, "row pairs of opposite column parities");

    // staging, every global load issued before the first LDS store
    constexpr int NX = LY * LX, NB = BY * BX;
    constexpr int IX = (NX + kSweep2xRestrictThreads - 1) / kSweep2xRestrictThreads;
    constexpr int IB = (NB + kSweep2xRestrictThreads - 1) / kSweep2xRestrictThreads;
    {
        T xv[IX], bv[IB];
#pragma unroll
        for (int t = 0; t < IX; ++t) {
            const int q = tid + t * kSweep2xRestrictThreads;
            T v = T(0);
            if (!ZERO_IN && q < NX) {
                const int ly = q / LX, lx = q - ly * LX;
                const int gi = x0 - H + lx, gj = y0 - H + ly;
                if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = xin[(int64_t)gj * g.nx + gi];
            }
            xv[t] = v;
        }
#pragma unroll
        for (int t = 0; t < IB; ++t) {
            const int q = tid + t * kSweep2xRestrictThreads;
            T v = T(0);
            if (q < NB) {
                const int ly = q / BX, lx = q - ly * BX;
                const int gi = x0 - BH + lx, gj = y0 - BH + ly;
                if (IN || (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)) v = b[(int64_t)gj * g.nx + gi];
            }
            bv[t] = v;
        }
#pragma unroll
        for (int t = 0; t < IX; ++t) {
            const int q = tid + t * kSweep2xRestrictThreads;
            if (q < NX) X[q] = xv[t];
        }
#pragma unroll
        for (int t = 0; t < IB; ++t) {
            const int q = tid + t * kSweep2xRestrictThreads;
            if (q < NB) B[q] = bscale * bv[t];
        }
    }
    __syncthreads();

    const T cxc = axis_coef<T, ORDER>(g.ihx2), cyc = axis_coef<T, ORDER>(g.ihy2);
    // L_h x at LDS cell p of global point (gi, gj) (the Dirichlet closure)
    auto lap = [&](int p, int gi, int gj, T uc) -> T {
        T dx, dy;
        if (ORDER == 2) {
            dx = X[p - 1] + X[p + 1] - T(2) * uc;
            dy = X[p - LX] + X[p + LX] - T(2) * uc;
        } else {
            const T l2 = (!IN && gi == 0) ? -uc : X[p - 2];
            const T r2 = (!IN && gi == g.nx - 1) ? -uc : X[p + 2];
            const T d2 = (!IN && gj == 0) ? -uc : X[p - 2 * LX];
            const T u2 = (!IN && gj == g.ny - 1) ? -uc : X[p + 2 * LX];
            dx = T(16) * (X[p - 1] + X[p + 1]) - (l2 + r2) - T(30) * uc;
            dy = T(16) * (X[p - LX] + X[p + LX]) - (d2 + u2) - T(30) * uc;
        }
        return dx * cxc + dy * cyc;
    };
    auto relax = [&](int gi, int gj) -> T {
        const int p = (gj - y0 + H) * LX + (gi - x0 + H);
        const T bval = B[(gj - y0 + BH) * BX + (gi - x0 + BH)];
        const T uc = X[p];
        const T r = bval - (uc - a * lap(p, gi, gj, uc));
        const bool edge = !IN && ORDER == 4 && (gi == 0 || gi == g.nx - 1 || gj == 0 || gj == g.ny - 1);
        return edge ? uc + (w * r) / mdiag_w<T, ORDER, 2>(gi, gj, 0, g, a, 0) : uc + r * inv_diag;
    };
    // one half-sweep of colour `colour` on the tile plus K layers, into LDS
    auto half = [&](auto kc, int colour) {
        constexpr int K = decltype(kc)::value;
        constexpr int W2 = (TX + 2 * K) / 2, NRW = TY + 2 * K, NP = NRW * W2;
        constexpr int IT = (NP + kSweep2xRestrictThreads - 1) / kSweep2xRestrictThreads;
        T rv[IT];
        int rp[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            rp[t] = -1;
            const int idx = tid + t * kSweep2xRestrictThreads;
            if (idx >= NP) continue;
            // lanes alternate between the two rows of a pair (bank-conflict
            // free reads, as in sweep_phases; the row count is even)
            const int pr = idx / (2 * W2), q2 = idx - pr * (2 * W2);
            const int r = 2 * pr + (q2 & 1), k2 = q2 >> 1;
            const int gj = y0 - K + r;
            const int gi = x0 - K + ((colour + gj + x0 - K) & 1) + 2 * k2;
            if (!IN && (gj < 0 || gj >= g.ny || gi < 0 || gi >= g.nx)) continue;
            rv[t] = relax(gi, gj);
            rp[t] = (gj - y0 + H) * LX + (gi - x0 + H);
        }
        if (ORDER == 4) __syncthreads();  // same-colour neighbours are read old (order 4 only)
#pragma unroll
        for (int t = 0; t < IT; ++t)
            if (rp[t] >= 0) X[rp[t]] = rv[t];
        __syncthreads();
    };
    half(std::integral_constant<int, M + 3>{}, 0);  // red, first sweep
    half(std::integral_constant<int, M + 2>{}, 1);  // black, first sweep
    half(std::integral_constant<int, M + 1>{}, 0);  // red, second sweep
    half(std::integral_constant<int, M>{}, 1);      // black, second sweep

    // the tile's new iterate
    for (int q = tid; q < TX * TY; q += kSweep2xRestrictThreads) {
        const int r = q / TX, c = q - r * TX;
        const int gi = x0 + c, gj = y0 + r;
        if (IN || (gi < g.nx && gj < g.ny)) xout[(int64_t)gj * g.nx + gi] = X[(r + H) * LX + c + H];
    }
    // residual over fine points [x0, x0 + 64] x [y0, y0 + TY] (0 outside the grid)
    constexpr int IR = (NR + kSweep2xRestrictThreads - 1) / kSweep2xRestrictThreads;
    T rv[IR];
#pragma unroll
    for (int t = 0; t < IR; ++t) {
        const int q = tid + t * kSweep2xRestrictThreads;
        T r = T(0);
        if (q < NR) {
            const int ry = q / RX, rx = q - ry * RX;
            const int gi = x0 + rx, gj = y0 + ry;
            if (IN || (gi < g.nx && gj < g.ny)) {
                const int p = (ry + H) * LX + rx + H;
                const T uc = X[p];
                r = B[(ry + BH) * BX + rx + BH] - (uc - a * lap(p, gi, gj, uc));
            }
        }
        rv[t] = r;
    }
    __syncthreads();  // every read of b is done: its LDS takes r
#pragma unroll
    for (int t = 0; t < IR; ++t) {
        const int q = tid + t * kSweep2xRestrictThreads;
        if (q < NR) B[q] = rv[t];
    }
    __syncthreads();
    // full weighting onto the coarse points of the tile
    for (int q = tid; q < (TX / 2) * (TY / 2); q += kSweep2xRestrictThreads) {
        const int cy = q / (TX / 2), cx = q - cy * (TX / 2);
        const int ic = (x0 >> 1) + cx, jc = (y0 >> 1) + cy;
        if (ic >= gc.nx || jc >= gc.ny) continue;
        const int fx = 2 * cx + 1, fy = 2 * cy + 1;
        T sum = T(0);
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            T row = T(0);
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) row += (ox == 0 ? T(0.5) : T(0.25)) * B[(fy + oy) * RX + fx + ox];
            sum += (oy == 0 ? T(0.5) : T(0.25)) * row;
        }
        bc[(int64_t)jc * gc.nx + ic] = sum;
    }
}

template <typename T, int ORDER, int TY, bool ZERO_IN>
__global__ __launch_bounds__(kSweep2xRestrictThreads) void k_sweep2x_restrict_tile2d(const T* __restrict__ xin,
                                                                          const T* __restrict__ b, T bscale,
                                                                          T* __restrict__ xout, Geo g, T a,
                                                                          T inv_diag, T w, T* __restrict__ bc,
                                                                          Geo gc) {
    constexpr int TX = 64;
    constexpr int R = ORDER / 2, M = R + 1, H = R + M + 3;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int BH = M + 3, BX = TX + 2 * BH, BY = TY + 2 * BH;
    __shared__ T X[LY * LX];
    __shared__ T B[BY * BX];
    const int tid = threadIdx.x;
    int bx, by;
    xcd_block(bx, by);  // XCD-contiguous bands of tiles
    const int x0 = bx * TX, y0 = by * TY;
    if (tile_inside2d(g, x0, x0 + TX, y0, y0 + TY, H))
        sweep2x_restrict_body<T, ORDER, TY, ZERO_IN, true>(xin, b, bscale, xout, g, a, inv_diag, w, bc, gc, X, B, tid,
                                                           x0, y0);
    else
        sweep2x_restrict_body<T, ORDER, TY, ZERO_IN, false>(xin, b, bscale, xout, g, a, inv_diag, w, bc, gc, X, B,
                                                            tid, x0, y0);
}

template <typename T, int ORDER, int TY>
static hipError_t sweep2x_restrict_launch(const T* xin, const T* b, T bs, T* xout, const Geo& g, T aa, T inv, T w,
                                          bool zero_in, T* bc, const Geo& gc, hipStream_t s, hipEvent_t ev0,
                                          hipEvent_t ev1) {
    dim3 grid((g.nx + 63) / 64, (g.ny + TY - 1) / TY, 1);
    dim3 block(kSweep2xRestrictThreads);
    if (zero_in)
        hipExtLaunchKernelGGL((k_sweep2x_restrict_tile2d<T, ORDER, TY, true>), grid, block, 0, s, ev0, ev1, 0, xin, b, bs, xout, g, aa, inv, w, bc, gc);
    else
        hipExtLaunchKernelGGL((k_sweep2x_restrict_tile2d<T, ORDER, TY, false>), grid, block, 0, s, ev0, ev1, 0, xin, b, bs, xout, g, aa, inv, w, bc, gc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep2x_restrict2d(const T* xin, const T* b, double bscale, T* xout, const Geo& g, int order,
                                     double a, double w, bool zero_in, T* bc, const Geo& gc, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    if (g.dim != 2 || g.wall || gc.nx != (g.nx - 1) / 2 || gc.ny != (g.ny - 1) / 2) return hipErrorInvalidValue;
    const double c0 = order == 2 ? 2.0 : 30.0 / 12.0;
    const T inv = (T)(w / (1.0 + a * c0 * (g.ihx2 + g.ihy2)));
    const T bs = (T)bscale, ww = (T)w, aa = (T)a;
    // the tile heights of the plain fused pre-smoothing
    const bool tall = (int64_t)((g.nx + 63) / 64) * ((g.ny + 15) / 16) >= 1024;
    if (order == 2)
        return tall ? sweep2x_restrict_launch<T, 2, 16>(xin, b, bs, xout, g, aa, inv, ww, zero_in, bc, gc, s, ev0, ev1)
                    : sweep2x_restrict_launch<T, 2, 8>(xin, b, bs, xout, g, aa, inv, ww, zero_in, bc, gc, s, ev0, ev1);
    return tall ? sweep2x_restrict_launch<T, 4, 16>(xin, b, bs, xout, g, aa, inv, ww, zero_in, bc, gc, s, ev0, ev1)
                : sweep2x_restrict_launch<T, 4, 8>(xin, b, bs, xout, g, aa, inv, ww, zero_in, bc, gc, s, ev0, ev1);
}

template hipError_t launch_sweep2x_restrict2d<double>(const double*, const double*, double, double*, const Geo&, int,
                                                      double, double, bool, double*, const Geo&, hipStream_t,
                                                      hipEvent_t, hipEvent_t);
template hipError_t launch_sweep2x_restrict2d<float>(const float*, const float*, double, float*, const Geo&, int,
                                                     double, double, bool, float*, const Geo&, hipStream_t,
                                                     hipEvent_t, hipEvent_t);

template <typename T>
hipError_t launch_sweep2d(const T* xin, const T* xc, const T* b, double bscale, T* xout, const Geo& g, const Geo& gc,
                          int order, double a, double w, bool zero_in, bool prolong, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
    const T bs = (T)bscale;
    if (order == 2) return sweep2d_dispatch<T, 2>(xin, xc, b, bs, xout, g, gc, a, w, zero_in, prolong, s, ev0, ev1);
    return sweep2d_dispatch<T, 4>(xin, xc, b, bs, xout, g, gc, a, w, zero_in, prolong, s, ev0, ev1);
}

template hipError_t launch_sweep2d<double>(const double*, const double*, const double*, double, double*, const Geo&,
                                           const Geo&, int, double, double, bool, bool, hipStream_t, hipEvent_t,
                                           hipEvent_t);
template hipError_t launch_sweep2d<float>(const float*, const float*, const float*, double, float*, const Geo&,
                                          const Geo&, int, double, double, bool, bool, hipStream_t, hipEvent_t,
                                          hipEvent_t);

}  // namespace ew
