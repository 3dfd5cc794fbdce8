// Explicit wave-solve on a small single curvilinear grid, several leapfrog
// steps per launch (Sec. "Discrete approximations": eqs. explicitStep1,
// explicitScheme and filterQuadrature with the order-2 mapped operator).
//
// On a grid of some 65k points one step moves under 5 MB, less than a launch
// costs, so the per-step kernel runs at the launch rate.  Here a workgroup
// stages a region of kRX x kRY points (its kTX x kTY output tile and a halo of
// kSteps points on each side) of both states and of the four coefficient
// arrays in LDS, then advances up to kSteps steps there: after step s only the
// points at least s + 1 from the region's edge are current, and after the
// last step the output tile still is.  The filter sum of the tile's points is
// kept in registers.  Every point update is the per-step kernel's expression
// on the same values, so the result is the same.  Tiles overlap in their
// halos, so a launch reads one pair of state arrays and writes the other.
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
constexpr int kThreads = 256;
constexpr int kPts = kRX * kRY / kThreads;  // region points per thread
static_assert(kRX * kRY % kThreads == 0, "region points split evenly over the threads");

// Grids up to this many points take the blocked kernel; above it the
// per-step kernel streams at most of the HBM rate.
constexpr int64_t kMaxBlockedPoints = int64_t(1) << 18;

// Steps k0 .. k0 + ns - 1 (1 <= ns <= kSteps), step k making W^{k+1} from
// W^k = wcur and W^{k-1} = wprev and adding cfil[k + 1] W^{k+1} to acc (with
// FIRST, k0 = 0: W^1 from W^0 alone, acc = cfil[0] W^0 + cfil[1] W^1).
// Writes W^{k0+ns} to dcur and W^{k0+ns-1} to dprev.
template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_leapfrog_mapped_blocked(
    const double* __restrict__ wcur, const double* __restrict__ wprev, double* __restrict__ dcur,
    double* __restrict__ dprev, double* __restrict__ acc, Geo g, MapCoef m, double dt2,
    const double* __restrict__ cfil, int k0, int ns) {
    __shared__ double sU[2][kRX * kRY];        // the two states, swapped each step
    __shared__ double sW[(kRX + 1) * kRY];     // A11 / dr^2 at half points x - 1/2 .. x + kRX - 1/2
    __shared__ double sS[kRX * (kRY + 1)];     // A22 / ds^2 at half points y - 1/2 .. y + kRY - 1/2
    __shared__ double sB[kRX * kRY];           // J a^12 / (4 dr ds), 0 beyond the walls
    __shared__ double sJ[kRX * kRY];           // 1 / J
    const int nx = g.nx, ny = g.ny;
    const int ox = (int)blockIdx.x * kTX - kSteps;  // grid coordinates of region point (0, 0)
    const int oy = (int)blockIdx.y * kTY - kSteps;
    const int t = threadIdx.x;

    int depth[kPts];     // distance to the region's edge, -1 beyond the walls
    double fsum[kPts];   // filter sum of an output point
#pragma unroll
    for (int q = 0; q < kPts; ++q) {
        const int p = t + q * kThreads;
        const int x = p % kRX, y = p / kRX;
        const int gx = ox + x, gy = oy + y;
        const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        const int d = std::min(std::min(x, kRX - 1 - x), std::min(y, kRY - 1 - y));
        const int64_t c = (int64_t)gy * nx + gx;
        sU[0][p] = in ? wcur[c] : 0.0;
        sU[1][p] = (!FIRST && in) ? wprev[c] : 0.0;
        sB[p] = in ? m.cb[c] : 0.0;
        sJ[p] = in ? m.ij[c] : 0.0;
        depth[q] = in ? d : -1;
        fsum[q] = (!FIRST && in && d >= kSteps) ? acc[c] : 0.0;
    }
    for (int p = t; p < (kRX + 1) * kRY; p += kThreads) {
        const int x = p % (kRX + 1), y = p / (kRX + 1);
        const int gx = ox + x, gy = oy + y;
        sW[p] = (gx >= 0 && gx <= nx && gy >= 0 && gy < ny) ? m.cw[(int64_t)gy * (nx + 1) + gx] : 0.0;
    }
    for (int p = t; p < kRX * (kRY + 1); p += kThreads) {
        const int x = p % kRX, y = p / kRX;
        const int gx = ox + x, gy = oy + y;
        sS[p] = (gx >= 0 && gx < nx && gy >= 0 && gy <= ny) ? m.cs[(int64_t)gy * nx + gx] : 0.0;
    }
    __syncthreads();

    int a = 0;  // sU[a] holds W^k, sU[a ^ 1] W^{k-1}
    for (int s = 0; s < ns; ++s) {
        const double* u = sU[a];
        double* un = sU[a ^ 1];
        const double cnext = cfil[k0 + s + 1];
#pragma unroll
        for (int q = 0; q < kPts; ++q) {
            if (depth[q] <= s) continue;  // not current after this step (or beyond a wall)
            const int p = t + q * kThreads;
            const int x = p % kRX, y = p / kRX;
            // L_h u as the per-step kernel forms it; values beyond the walls are 0
            const double uc = u[p];
            const double uW = u[p - 1], uE = u[p + 1], uS = u[p - kRX], uN = u[p + kRX];
            const double uSW = u[p - kRX - 1], uSE = u[p - kRX + 1];
            const double uNW = u[p + kRX - 1], uNE = u[p + kRX + 1];
            const int hw = y * (kRX + 1) + x;
            double tt = sW[hw + 1] * (uE - uc) - sW[hw] * (uc - uW);
            tt += sS[p + kRX] * (uN - uc) - sS[p] * (uc - uS);
            const double bE = sB[p + 1], bW = sB[p - 1], bN = sB[p + kRX], bS = sB[p - kRX];
            tt += bE * (uNE - uSE) - bW * (uNW - uSW);
            tt += bN * (uNE - uNW) - bS * (uSE - uSW);
            const double lap = sJ[p] * tt;
            double wn;
            if (FIRST && s == 0) {
                wn = uc + (0.5 * dt2) * lap;
                fsum[q] = cfil[0] * uc + cnext * wn;
            } else {
                wn = 2.0 * uc - un[p] + dt2 * lap;
                fsum[q] = fsum[q] + cnext * wn;
            }
            un[p] = wn;  // only this thread reads un[p] in this step
        }
        a ^= 1;
        __syncthreads();
    }

#pragma unroll
    for (int q = 0; q < kPts; ++q) {
        if (depth[q] < kSteps) continue;
        const int p = t + q * kThreads;
        const int64_t c = (int64_t)(oy + p / kRX) * nx + (ox + p % kRX);
        dcur[c] = sU[a][p];
        dprev[c] = sU[a ^ 1][p];
        acc[c] = fsum[q];
    }
}

}  // namespace

bool mapped_steps_blocked(const Geo& g) { return g.dim == 2 && g.size() <= kMaxBlockedPoints; }

int mapped_steps_per_launch() { return kSteps; }

hipError_t launch_leapfrog_mapped_blocked(const double* wcur, const double* wprev, double* dcur, double* dprev,
                                          double* acc, const Geo& g, const MapCoef& m, double dt2,
                                          const double* cfil_dev, int k0, int ns, hipStream_t s) {
    if (ns < 1 || ns > kSteps || k0 < 0 || (k0 == 0) != (wprev == nullptr) || !mapped_steps_blocked(g))
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
