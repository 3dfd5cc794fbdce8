// Explicit wave-solve on a 2D box in FP64, several leapfrog steps per launch
// (eqs. explicitStep1, explicitScheme and filterQuadrature with the order-2
// or order-4 operator of eq. eigBVPdiscrete and its wall closures).
//
// One launch per step streams 40 B per point-step.  Here a workgroup loads a
// 32 x 32 region (its 16 x 16 output tile and a halo of 8 points), then
// advances up to 8 / R steps on it, R the stencil's radius (1 for order 2,
// 2 for order 4): after step s only the points at least R (s + 1) from the
// region's edge are current, and after the last step the output tile still
// is.  The current state is shared through LDS (two buffers, swapped each
// step; points beyond the walls read 0 there and the closures of d2_framed
// replace them), each point's previous state and filter sum stay in its
// thread's registers.  Every update is the per-step kernel's expression on
// the same values.  Tiles overlap in their halos, so a launch reads one pair
// of state arrays and writes the other.
#include "op.h"
#include "stencil_dev.h"

namespace ew {

namespace {

constexpr int kTX = 16;  // output tile
constexpr int kTY = 16;
constexpr int kHalo = 8;
constexpr int kRX = kTX + 2 * kHalo;
constexpr int kRY = kTY + 2 * kHalo;
constexpr int kThreads = kRX * kRY;  // one region point per thread
static_assert(kThreads <= 1024, "one workgroup covers the region");

template <int ORDER>
constexpr int steps_per_launch() {
    return kHalo / (ORDER / 2);
}

// Steps k0 .. k0 + ns - 1 (1 <= ns <= steps_per_launch), step k making
// W^{k+1} from W^k = wcur and W^{k-1} = wprev and adding cfil[k + 1] W^{k+1}
// to acc (with FIRST, k0 = 0: W^1 from W^0 alone, acc = cfil[0] W^0 +
// cfil[1] W^1).  Writes W^{k0+ns} to dcur and W^{k0+ns-1} to dprev.
template <int ORDER, bool FIRST>
__global__ __launch_bounds__(kThreads) void k_leapfrog_box_blocked(const double* __restrict__ wcur,
                                                                   const double* __restrict__ wprev,
                                                                   double* __restrict__ dcur, double* __restrict__ dprev,
                                                                   double* __restrict__ acc, Geo g, double dt2,
                                                                   const double* __restrict__ cfil, int k0, int ns) {
    constexpr int kR = ORDER / 2;
    constexpr int kSteps = steps_per_launch<ORDER>();
    __shared__ double sU[2][kRX * kRY];  // the current state, double-buffered across a step
    __shared__ double sC[kSteps + 1];    // the launch's filter weights cfil[k0 .. k0 + ns]
    const int nx = g.nx, ny = g.ny;
    const int t = threadIdx.x;
    const int x = t % kRX, y = t / kRX, p = t;
    const int gx = (int)blockIdx.x * kTX - kHalo + x;
    const int gy = (int)blockIdx.y * kTY - kHalo + y;
    const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int depth = min(min(x, kRX - 1 - x), min(y, kRY - 1 - y));
    const int64_t c = (int64_t)gy * nx + gx;
    // current after steps 0 .. last - 1 (never beyond a wall)
    const int last = in ? depth / kR : 0;
    double cur = in ? wcur[c] : 0.0;
    double prv = (!FIRST && in) ? wprev[c] : 0.0;
    double fsum = (!FIRST && in && depth >= kHalo) ? acc[c] : 0.0;
    sU[0][p] = cur;
    sU[1][p] = 0.0;  // beyond the walls both buffers must read 0
    if (t <= ns) sC[t] = cfil[k0 + t];
    const double cx = axis_coef<double, ORDER>(g.ihx2), cy = axis_coef<double, ORDER>(g.ihy2);
    const int wx = g.wall & 3, wy = (g.wall >> 2) & 3;
    __syncthreads();

#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        if (s >= ns) break;
        const double* u = sU[s & 1];  // W^{k0+s}
        double* un = sU[(s & 1) ^ 1];
        if (last > s) {
            // L_h u as lap_at forms it, from the frame
            const double uc = cur;
            double lap = d2_framed<double, ORDER>(u, p, 1, gx, nx, uc, wx) * cx;
            lap += d2_framed<double, ORDER>(u, p, kRX, gy, ny, uc, wy) * cy;
            const double cnext = sC[s + 1];
            double wn;
            if (FIRST && s == 0) {
                wn = uc + (0.5 * dt2) * lap;
                fsum = sC[0] * uc + cnext * wn;
            } else {
                wn = 2.0 * uc - prv + dt2 * lap;
                fsum = fsum + cnext * wn;
            }
            prv = cur;
            cur = wn;
            un[p] = wn;  // only this thread reads un[p] in this step
        }
        __syncthreads();
    }

    if (in && depth >= kHalo) {
        dcur[c] = cur;
        dprev[c] = prv;
        acc[c] = fsum;
    }
}

}  // namespace

int box_steps_per_launch(int order) { return order == 2 ? steps_per_launch<2>() : steps_per_launch<4>(); }

hipError_t launch_leapfrog_box_blocked(const double* wcur, const double* wprev, double* dcur, double* dprev,
                                       double* acc, const Geo& g, int order, double dt2, const double* cfil_dev,
                                       int k0, int ns, hipStream_t s) {
    if ((order != 2 && order != 4) || g.dim != 2 || ns < 1 || ns > box_steps_per_launch(order) || k0 < 0 ||
        (k0 == 0) != (wprev == nullptr))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((g.nx + kTX - 1) / kTX), (unsigned)((g.ny + kTY - 1) / kTY), 1);
#define EW_BOX_LF(O)                                                                                             \
    do {                                                                                                         \
        if (k0 == 0)                                                                                             \
            k_leapfrog_box_blocked<O, true><<<grid, kThreads, 0, s>>>(wcur, wprev, dcur, dprev, acc, g, dt2,     \
                                                                      cfil_dev, k0, ns);                         \
        else                                                                                                     \
            k_leapfrog_box_blocked<O, false><<<grid, kThreads, 0, s>>>(wcur, wprev, dcur, dprev, acc, g, dt2,    \
                                                                       cfil_dev, k0, ns);                        \
    } while (0)
    if (order == 2) EW_BOX_LF(2);
    else EW_BOX_LF(4);
#undef EW_BOX_LF
    return hipGetLastError();
}

}  // namespace ew
