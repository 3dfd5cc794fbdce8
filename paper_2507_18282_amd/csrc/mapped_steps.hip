// Explicit wave-solve on a single curvilinear grid, several leapfrog steps
// per launch (Sec. "Discrete approximations": eqs. explicitStep1,
// explicitScheme and filterQuadrature with the order-2 mapped operator).
//
// One launch per step streams 72 B per point-step (two states, the filter
// sum and four coefficient arrays) and, on small grids, costs more than the
// data it moves.  Here a workgroup loads a region of kRX x kRY points (its
// kTX x kTY output tile and a halo of kSteps points on each side), then
// advances up to kSteps steps on it: after step s only the points at least
// s + 1 from the region's edge are current, and after the last step the
// output tile still is.  The current state is shared through LDS; each
// point's previous state, coefficients and (in the output tile) filter sum
// stay in its thread's registers.  Every point update is the per-step
// expression on the same values, so the result does not depend on kSteps.
// Tiles overlap in their halos, so a launch reads one pair of state arrays
// and writes the other.  Against one launch per step (which streamed at 0.84
// of the HBM peak on 2047^2) a wave-solve took 0.187 against 0.725 ms on
// 255^2, 1.93 against 3.33 ms on 1023^2 and 14.2 against 22.3 ms on 2047^2.
#include <algorithm>

#include "op.h"
#include "stencil_dev.h"

namespace ew {

namespace {

constexpr int kTX = 16;     // output tile
constexpr int kTY = 16;
constexpr int kSteps = 8;   // steps per launch and halo width
constexpr int kRX = kTX + 2 * kSteps;
constexpr int kRY = kTY + 2 * kSteps;
// Consecutive rows of one column per thread.  A step is bound by latency
// (LDS reads, a chain of FP64 operations and the barrier), not by LDS or
// arithmetic throughput, so more wavefronts per CU hide more of it: on a
// 255^2 annulus (191 steps) a wave-solve took 0.246, 0.204 and 0.187 ms
// with strips of 4, 2 and 1 rows (256, 512 and 1024 threads), and 0.202 ms
// with 16 steps per launch and strips of 3.
constexpr int kStrip = 1;
constexpr int kThreads = kRX * kRY / kStrip;
static_assert(kRY % kStrip == 0, "threads cover the region in strips");

// Steps k0 .. k0 + ns - 1 (1 <= ns <= kSteps), step k making W^{k+1} from
// W^k = wcur and W^{k-1} = wprev and adding cfil[k + 1] W^{k+1} to acc (with
// FIRST, k0 = 0: W^1 from W^0 alone, acc = cfil[0] W^0 + cfil[1] W^1).
// Writes W^{k0+ns} to dcur and W^{k0+ns-1} to dprev.
//
// Each thread owns a strip of kStrip rows of one region column and keeps
// their previous states and their nine coefficients in registers; a step
// reads from LDS only the two side columns beside the strip and the points
// just below and above it, and writes the strip's new values for the
// neighbours.
template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_leapfrog_mapped_blocked(
    const double* __restrict__ wcur, const double* __restrict__ wprev, double* __restrict__ dcur,
    double* __restrict__ dprev, double* __restrict__ acc, Geo g, MapCoef m, double dt2,
    const double* __restrict__ cfil, int k0, int ns) {
    __shared__ double sU[2][kRX * kRY];  // the current state, double-buffered across a step
    __shared__ double sC[kSteps + 1];    // the launch's filter weights cfil[k0 .. k0 + ns]
    const int nx = g.nx, ny = g.ny;
    const int ox = (int)blockIdx.x * kTX - kSteps;  // grid coordinates of region point (0, 0)
    const int oy = (int)blockIdx.y * kTY - kSteps;
    const int t = threadIdx.x;
    const int x = t % kRX;
    const int y0 = (t / kRX) * kStrip;  // first row of the strip
    const int gx = ox + x;

    if (t <= ns) sC[t] = cfil[k0 + t];  // read once, ahead of the step chain
    int depth[kStrip];   // distance to the region's edge, -1 beyond the walls
    double cur[kStrip], prv[kStrip], fsum[kStrip];
    // the strip's coefficients, as the per-step kernel reads them (used only
    // at points that are ever updated, which lie inside the grid)
    double kw[kStrip], ke[kStrip], ks[kStrip], kn[kStrip];
    double bw[kStrip], be[kStrip], bs[kStrip], bn[kStrip], kj[kStrip];
#pragma unroll
    for (int q = 0; q < kStrip; ++q) {
        const int y = y0 + q, p = y * kRX + x;
        const int gy = oy + y;
        const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        const int d = std::min(std::min(x, kRX - 1 - x), std::min(y, kRY - 1 - y));
        const int64_t c = (int64_t)gy * nx + gx;
        const int64_t hw = (int64_t)gy * (nx + 1) + gx;  // half point gx - 1/2
        cur[q] = in ? wcur[c] : 0.0;
        prv[q] = (!FIRST && in) ? wprev[c] : 0.0;
        sU[0][p] = cur[q];
        sU[1][p] = 0.0;  // beyond the walls both buffers must read 0
        depth[q] = in ? d : -1;
        fsum[q] = (!FIRST && in && d >= kSteps) ? acc[c] : 0.0;
        kw[q] = in ? m.cw[hw] : 0.0;
        ke[q] = in ? m.cw[hw + 1] : 0.0;
        ks[q] = in ? m.cs[c] : 0.0;
        kn[q] = in ? m.cs[c + nx] : 0.0;
        bw[q] = in && gx > 0 ? m.cb[c - 1] : 0.0;
        be[q] = in && gx < nx - 1 ? m.cb[c + 1] : 0.0;
        bs[q] = in && gy > 0 ? m.cb[c - nx] : 0.0;
        bn[q] = in && gy < ny - 1 ? m.cb[c + nx] : 0.0;
        kj[q] = in ? m.ij[c] : 0.0;
    }
    __syncthreads();

#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        if (s >= ns) break;
        const double* u = sU[s & 1];  // W^{k0+s}
        double* un = sU[(s & 1) ^ 1];
        const double cnext = sC[s + 1];
        bool act[kStrip];
        bool any = false;
#pragma unroll
        for (int q = 0; q < kStrip; ++q) {
            act[q] = depth[q] > s;  // current after this step (never beyond a wall)
            any = any || act[q];
        }
        if (any) {
            // an updated point has 1 <= x <= kRX - 2; rows y0 - 1 .. y0 + kStrip
            // outside the region are never a neighbour of one
            double lc[kStrip + 2], rc[kStrip + 2];
#pragma unroll
            for (int r = 0; r < kStrip + 2; ++r) {
                const int y = y0 - 1 + r;
                const bool ok = y >= 0 && y < kRY;
                lc[r] = ok ? u[y * kRX + x - 1] : 0.0;
                rc[r] = ok ? u[y * kRX + x + 1] : 0.0;
            }
            const double below = y0 >= 1 ? u[(y0 - 1) * kRX + x] : 0.0;
            const double above = y0 + kStrip < kRY ? u[(y0 + kStrip) * kRX + x] : 0.0;
            double nxt[kStrip], nfs[kStrip];
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                // L_h u as the per-step kernel forms it; values beyond the walls are 0
                const double uc = cur[q];
                const double uS = q > 0 ? cur[q - 1] : below;
                const double uN = q < kStrip - 1 ? cur[q + 1] : above;
                const double uW = lc[q + 1], uE = rc[q + 1];
                const double uSW = lc[q], uSE = rc[q], uNW = lc[q + 2], uNE = rc[q + 2];
                double tt = ke[q] * (uE - uc) - kw[q] * (uc - uW);
                tt += kn[q] * (uN - uc) - ks[q] * (uc - uS);
                tt += be[q] * (uNE - uSE) - bw[q] * (uNW - uSW);
                tt += bn[q] * (uNE - uNW) - bs[q] * (uSE - uSW);
                const double lap = kj[q] * tt;
                double wn;
                if (FIRST && s == 0) {
                    wn = uc + (0.5 * dt2) * lap;
                    nfs[q] = sC[0] * uc + cnext * wn;
                } else {
                    wn = 2.0 * uc - prv[q] + dt2 * lap;
                    nfs[q] = fsum[q] + cnext * wn;
                }
                nxt[q] = wn;
            }
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                if (!act[q]) continue;
                fsum[q] = nfs[q];
                prv[q] = cur[q];
                cur[q] = nxt[q];
                un[(y0 + q) * kRX + x] = nxt[q];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int q = 0; q < kStrip; ++q) {
        if (depth[q] < kSteps) continue;
        const int64_t c = (int64_t)(oy + y0 + q) * nx + gx;
        dcur[c] = cur[q];
        dprev[c] = prv[q];
        acc[c] = fsum[q];
    }
}

}  // namespace

int mapped_steps_per_launch() { return kSteps; }

hipError_t launch_leapfrog_mapped_blocked(const double* wcur, const double* wprev, double* dcur, double* dprev,
                                          double* acc, const Geo& g, const MapCoef& m, double dt2,
                                          const double* cfil_dev, int k0, int ns, hipStream_t s) {
    if (ns < 1 || ns > kSteps || k0 < 0 || (k0 == 0) != (wprev == nullptr) || g.dim != 2)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((g.nx + kTX - 1) / kTX), (unsigned)((g.ny + kTY - 1) / kTY), 1);
    if (k0 == 0)
        k_leapfrog_mapped_blocked<true><<<grid, kThreads, 0, s>>>(wcur, wprev, dcur, dprev, acc, g, m, dt2, cfil_dev,
                                                                  k0, ns);
    else
        k_leapfrog_mapped_blocked<false><<<grid, kThreads, 0, s>>>(wcur, wprev, dcur, dprev, acc, g, m, dt2,
                                                                   cfil_dev, k0, ns);
    return hipGetLastError();
}

}  // namespace ew
