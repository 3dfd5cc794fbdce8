// Kernels of the batched form: many independent Dirichlet rectangles advanced
// together, explicit leapfrog with the filter accumulated in the state type
// (FP32, or FP64 for k_batch_step).
//
//  * k_batch_small   one 1024-thread workgroup per small problem runs the
//                    whole wave-solve (all N_t steps) with W^n resident in LDS
//                    and W^{n-1} and the accumulator in registers: the
//                    problem never touches HBM between reading v and writing
//                    S v.
//  * k_batch_step    one leapfrog step (fused with the filter accumulation)
//                    for every large problem that still has steps left, in
//                    one launch; each workgroup reads its (problem, tile)
//                    from a table built on the host.
//  * k_batch_convert FP64 <-> FP32 copies of the boundary vectors.
//  * k_batch_mgs     one modified Gram-Schmidt link for every problem of a
//                    batched Arnoldi step (FP64), partial sums per problem.
#include "batch.h"
#include "stencil_dev.h"

namespace ew {

__device__ __forceinline__ int find_segment(const int* __restrict__ starts, int nseg, int b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // last segment whose start <= b
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------------------------
// Small problems: whole wave-solve in one workgroup.
// --------------------------------------------------------------------------
template <int ORDER>
__device__ __forceinline__ float lap_small(const float* X, int px, int p, int i, int j, int nx, int ny, float uc,
                                           float cx, float cy) {
    if (ORDER == 2) {
        return (X[p - 1] + X[p + 1] - 2.0f * uc) * cx + (X[p - px] + X[p + px] - 2.0f * uc) * cy;
    } else {
        const float l2 = (i == 0) ? -uc : X[p - 2], r2 = (i == nx - 1) ? -uc : X[p + 2];
        const float d2 = (j == 0) ? -uc : X[p - 2 * px], u2 = (j == ny - 1) ? -uc : X[p + 2 * px];
        const float dx = 16.0f * (X[p - 1] + X[p + 1]) - (l2 + r2) - 30.0f * uc;
        const float dy = 16.0f * (X[p - px] + X[p + px]) - (d2 + u2) - 30.0f * uc;
        return dx * cx + dy * cy;
    }
}

template <int ORDER>
__global__ __launch_bounds__(kBatchSmallThreads) void k_batch_small(BatchProbDev* __restrict__ probs,
                                                                    const int* __restrict__ small_ids,
                                                                    const float* __restrict__ coef) {
    extern __shared__ __align__(16) float Xs[];
    const BatchProbDev P = probs[small_ids[blockIdx.x]];
    if (!P.active) return;
    const Geo g = P.g;
    const int nx = g.nx, ny = g.ny, px = nx + 4;
    const int n = nx * ny;
    const int tid = threadIdx.x;
    const float cx = ORDER == 2 ? (float)g.ihx2 : (float)(g.ihx2 / 12.0);
    const float cy = ORDER == 2 ? (float)g.ihy2 : (float)(g.ihy2 / 12.0);
    const float dt2 = (float)P.dt2;
    const float* c = coef + P.coef_off;
    for (int q = tid; q < px * (ny + 4); q += kBatchSmallThreads) Xs[q] = 0.0f;
    __syncthreads();
    float cur[kBatchSmallPts], prev[kBatchSmallPts], acc[kBatchSmallPts];
    int lp[kBatchSmallPts], li[kBatchSmallPts], lj[kBatchSmallPts];
#pragma unroll
    for (int t = 0; t < kBatchSmallPts; ++t) {
        const int q = tid + t * kBatchSmallThreads;
        lp[t] = -1;
        if (q < n) {
            li[t] = q % nx;
            lj[t] = q / nx;
            lp[t] = (lj[t] + 2) * px + li[t] + 2;
            cur[t] = (float)P.v[q];
            Xs[lp[t]] = cur[t];
            acc[t] = c[0] * cur[t];
        }
    }
    __syncthreads();
    float nw[kBatchSmallPts];
    for (int step = 0; step < P.n_t; ++step) {
        const float cn = c[step + 1];
#pragma unroll
        for (int t = 0; t < kBatchSmallPts; ++t) {
            if (lp[t] < 0) continue;
            const float lap = lap_small<ORDER>(Xs, px, lp[t], li[t], lj[t], nx, ny, cur[t], cx, cy);
            nw[t] = (step == 0) ? cur[t] + (0.5f * dt2) * lap : 2.0f * cur[t] - prev[t] + dt2 * lap;
            acc[t] = acc[t] + cn * nw[t];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kBatchSmallPts; ++t) {
            if (lp[t] < 0) continue;
            Xs[lp[t]] = nw[t];
            prev[t] = cur[t];
            cur[t] = nw[t];
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < kBatchSmallPts; ++t) {
        const int q = tid + t * kBatchSmallThreads;
        if (q < n) P.out[q] = (double)acc[t];
    }
}

// --------------------------------------------------------------------------
// Large problems: one step for every problem, tiles of 64 x (4 TYR) points.
// --------------------------------------------------------------------------
template <int ORDER, int TYR, typename T>
__global__ __launch_bounds__(256) void k_batch_step(BatchProbDev* __restrict__ probs,
                                                    const BatchBlk* __restrict__ blk, const T* __restrict__ coef,
                                                    int step) {
    int wb, wy, wz;
    xcd_block(wb, wy, wz);  // each XCD takes a contiguous run of tiles (rows of a problem share halos)
    const BatchBlk bt = blk[wb];  // one load (a binary search over the problems' first tiles took seven)
    const BatchProbDev& P = probs[bt.prob];
    if (!P.active || step >= P.n_t) return;
    const Geo g = P.g;
    const int tiles_x = (g.nx + 63) >> 6;
    const int tile = bt.tile;
    const int i = (tile % tiles_x) * 64 + (threadIdx.x & 63);
    const int j0 = (tile / tiles_x) * (4 * TYR) + (threadIdx.x >> 6);
    if (i >= g.nx) return;
    // time level slots: W^0 in f0, odd levels in fA, even levels >= 2 in fB
    const T* f0 = static_cast<const T*>(P.f0);
    T* fA = static_cast<T*>(P.fA);
    T* fB = static_cast<T*>(P.fB);
    T* acc = static_cast<T*>(P.acc);
    const T* wcur = step == 0 ? f0 : ((step & 1) ? fA : fB);
    const T* wprev = step == 1 ? f0 : ((step & 1) ? fB : fA);
    T* wnext = ((step + 1) & 1) ? fA : fB;
    const T dt2 = (T)P.dt2;
    const T c0 = coef[P.coef_off], cn = coef[P.coef_off + step + 1];
#pragma unroll
    for (int r = 0; r < TYR; ++r) {
        const int j = j0 + 4 * r;
        if (j >= g.ny) break;
        const int64_t cidx = (int64_t)j * g.nx + i;
        const T uc = wcur[cidx];
        const T lap = lap_at<T, ORDER, 2, false>(wcur, cidx, i, j, 0, g, uc);
        T wn;
        if (step == 0) {
            wn = uc + ((T)0.5 * dt2) * lap;
            acc[cidx] = c0 * uc + cn * wn;
        } else {
            wn = (T)2 * uc - wprev[cidx] + dt2 * lap;
            acc[cidx] = acc[cidx] + cn * wn;
        }
        wnext[cidx] = wn;
    }
}

// --------------------------------------------------------------------------
// FP64 state: several steps per launch.  A workgroup loads a 32 x 32 region
// of one problem (its 16 x 16 output tile and an 8-point halo) and advances
// up to 8 / R steps on it (R the stencil's radius): after step s only the
// points at least R (s + 1) from the region's edge are current, and after the
// last step the output tile still is.  The current level is shared through
// LDS (two buffers; beyond the walls both read 0), each point's previous
// level and filter sum stay in registers; every update is k_batch_step's
// expression on the same values.
// --------------------------------------------------------------------------
constexpr int kBlkTile = 16;
constexpr int kBlkHalo = 8;
constexpr int kBlkSide = kBlkTile + 2 * kBlkHalo;
constexpr int kBlkThreads = kBlkSide * kBlkSide;  // one region point per thread

template <int ORDER>
__global__ __launch_bounds__(kBlkThreads) void k_batch_blocked(BatchProbDev* __restrict__ probs,
                                                               const BatchBlk* __restrict__ blk,
                                                               const double* __restrict__ coef, int launch) {
    constexpr int kR = ORDER / 2;
    constexpr int kSteps = kBlkHalo / kR;
    __shared__ double sU[2][kBlkThreads];
    __shared__ double sC[kSteps + 1];  // the launch's filter weights
    const BatchBlk bt = blk[blockIdx.x];
    const BatchProbDev& P = probs[bt.prob];
    const int k0 = launch * kSteps;
    if (!P.active || k0 >= P.n_t) return;  // the whole workgroup, before any barrier
    const int ns = min(kSteps, P.n_t - k0);
    const Geo g = P.g;
    const int nx = g.nx, ny = g.ny;
    const int tiles_x = (nx + kBlkTile - 1) / kBlkTile;
    const int t = threadIdx.x;
    const int x = t % kBlkSide, y = t / kBlkSide;
    const int gx = (bt.tile % tiles_x) * kBlkTile - kBlkHalo + x;
    const int gy = (bt.tile / tiles_x) * kBlkTile - kBlkHalo + y;
    const bool first = k0 == 0;
    const bool odd = (launch & 1) != 0;
    const double* wcur = static_cast<const double*>(first ? P.f0 : (odd ? P.fA : P.fC));
    const double* wprev = static_cast<const double*>(odd ? P.fB : P.fD);
    double* dcur = static_cast<double*>(odd ? P.fC : P.fA);
    double* dprev = static_cast<double*>(odd ? P.fD : P.fB);
    double* acc = static_cast<double*>(P.acc);
    const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int depth = min(min(x, kBlkSide - 1 - x), min(y, kBlkSide - 1 - y));
    const int64_t c = (int64_t)gy * nx + gx;
    const int last = in ? depth / kR : 0;  // current after steps 0 .. last - 1
    double cur = in ? wcur[c] : 0.0;
    double prv = (!first && in) ? wprev[c] : 0.0;
    double fsum = (!first && in && depth >= kBlkHalo) ? acc[c] : 0.0;
    sU[0][t] = cur;
    sU[1][t] = 0.0;
    if (t <= ns) sC[t] = coef[P.coef_off + k0 + t];
    const double cx = axis_coef<double, ORDER>(g.ihx2), cy = axis_coef<double, ORDER>(g.ihy2);
    const double dt2 = P.dt2;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        if (s >= ns) break;
        const double* u = sU[s & 1];
        double* un = sU[(s & 1) ^ 1];
        if (last > s) {
            const double uc = cur;
            double lap = d2_framed<double, ORDER>(u, t, 1, gx, nx, uc, 0) * cx;
            lap += d2_framed<double, ORDER>(u, t, kBlkSide, gy, ny, uc, 0) * cy;
            const double cn = sC[s + 1];
            double wn;
            if (first && s == 0) {
                wn = uc + (0.5 * dt2) * lap;
                fsum = sC[0] * uc + cn * wn;
            } else {
                wn = 2.0 * uc - prv + dt2 * lap;
                fsum = fsum + cn * wn;
            }
            prv = cur;
            cur = wn;
            un[t] = wn;
        }
        __syncthreads();
    }
    if (in && depth >= kBlkHalo) {
        dcur[c] = cur;
        dprev[c] = prv;
        acc[c] = fsum;
    }
}

// --------------------------------------------------------------------------
// FP64 <-> FP32 for the large problems (v -> f0 before the steps, acc -> out after).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_convert(BatchProbDev* __restrict__ probs, const int* __restrict__ ids,
                                                       const int* __restrict__ blk_start, int nseg, int to_fp32) {
    const int s = find_segment(blk_start, nseg, blockIdx.x);
    const BatchProbDev& P = probs[ids[s]];
    if (!P.active) return;
    const int64_t n = P.g.size();
    const int64_t base = (int64_t)(blockIdx.x - blk_start[s]) * (256 * kConvPerThread) + threadIdx.x;
#pragma unroll
    for (int t = 0; t < kConvPerThread; ++t) {
        const int64_t q = base + 256 * t;
        if (q >= n) break;
        if (to_fp32) static_cast<float*>(P.f0)[q] = (float)P.v[q];
        else P.out[q] = (double)static_cast<const float*>(P.acc)[q];
    }
}

// --------------------------------------------------------------------------
// Batched modified Gram-Schmidt link (FP64): for every problem with link
// `ell` <= its chain length, the same arithmetic as k_mgs_link / k_normalize.
// Link 0 starts (w, u_0); links 1..q-1 finish h_{ell-1}, subtract it and start
// the next product; link q-1 starts ||w||^2 (u_q = w); link q normalises.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_mgs(const BatchMgsDev* __restrict__ info, const MgsLink* __restrict__ links,
                                                   int nprob, const int* __restrict__ blk_start, int ell,
                                                   double* __restrict__ partial, double* __restrict__ hout) {
    const int s = find_segment(blk_start, nprob, blockIdx.x);
    const BatchMgsDev& I = info[s];
    if (ell > I.q) return;
    const int nb = blk_start[s + 1] - blk_start[s];
    const int b = blockIdx.x - blk_start[s];
    double* w = I.w;
    const int64_t n = I.n;
    double* pin = partial + I.part_off + ((ell + 1) & 1) * I.nblk;
    double* pout = partial + I.part_off + (ell & 1) * I.nblk;
    __shared__ double hsh;
    double h = 0.0;
    if (ell > 0) {
        double v = 0.0;
        for (int t = threadIdx.x; t < nb; t += 256) v += pin[t];
        const double r = block_sum_256(v, threadIdx.x);
        if (threadIdx.x == 0) hsh = r;
        __syncthreads();
        h = hsh;
        if (b == 0 && threadIdx.x == 0) hout[I.h_off + ell - 1] = (ell == I.q) ? sqrt(h) : h;
    }
    if (ell == I.q) {  // normalise
        const double nrm = sqrt(h);
        for (int64_t c = (int64_t)b * 256 + threadIdx.x; c < n; c += (int64_t)nb * 256) w[c] = w[c] / nrm;
        return;
    }
    const double* vprev = (ell > 0) ? links[(size_t)(ell - 1) * nprob + s].u : nullptr;
    const double* vnext = (ell < I.q - 1) ? links[(size_t)ell * nprob + s].u : w;
    const bool self = (vnext == w);
    double acc = 0.0;
    for (int64_t c = (int64_t)b * 256 + threadIdx.x; c < n; c += (int64_t)nb * 256) {
        double wi = w[c];
        if (ell > 0) {
            wi = wi - h * vprev[c];
            w[c] = wi;
        }
        acc += wi * (self ? wi : vnext[c]);
    }
    const double sum = block_sum_256(acc, threadIdx.x);
    if (threadIdx.x == 0) pout[b] = sum;
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
hipError_t launch_batch_small(BatchProbDev* probs, const int* small_ids, int nsmall, const float* coef, int order,
                              size_t lds_bytes, hipStream_t s) {
    if (nsmall == 0) return hipSuccess;
    if (order == 2) k_batch_small<2><<<nsmall, kBatchSmallThreads, lds_bytes, s>>>(probs, small_ids, coef);
    else k_batch_small<4><<<nsmall, kBatchSmallThreads, lds_bytes, s>>>(probs, small_ids, coef);
    return hipGetLastError();
}

hipError_t prepare_batch_small(int order, size_t lds_bytes) {
    const void* f = order == 2 ? (const void*)k_batch_small<2> : (const void*)k_batch_small<4>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

template <typename T>
static void batch_step_typed(BatchProbDev* probs, const BatchBlk* blk, int nblocks, const T* coef, int step,
                             int order, int tyr, hipStream_t s) {
#define EW_BSTEP(O, R) k_batch_step<O, R, T><<<nblocks, 256, 0, s>>>(probs, blk, coef, step)
    if (order == 2) {
        switch (tyr) { case 1: EW_BSTEP(2, 1); break; case 2: EW_BSTEP(2, 2); break; case 4: EW_BSTEP(2, 4); break; default: EW_BSTEP(2, 8); }
    } else {
        switch (tyr) { case 1: EW_BSTEP(4, 1); break; case 2: EW_BSTEP(4, 2); break; case 4: EW_BSTEP(4, 4); break; default: EW_BSTEP(4, 8); }
    }
#undef EW_BSTEP
}

hipError_t launch_batch_step(BatchProbDev* probs, const BatchBlk* blk, int nblocks, const void* coef, int step,
                             int order, int tyr, int fp64, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    if (fp64)
        batch_step_typed<double>(probs, blk, nblocks, static_cast<const double*>(coef), step, order, tyr, s);
    else
        batch_step_typed<float>(probs, blk, nblocks, static_cast<const float*>(coef), step, order, tyr, s);
    return hipGetLastError();
}

int batch_steps_per_launch(int order) { return kBlkHalo / (order / 2); }

int batch_blocked_tiles(const Geo& g) {
    return ((g.nx + kBlkTile - 1) / kBlkTile) * ((g.ny + kBlkTile - 1) / kBlkTile);
}

hipError_t launch_batch_blocked(BatchProbDev* probs, const BatchBlk* blk, int nblocks, const double* coef, int launch,
                                int order, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    if (order == 2) k_batch_blocked<2><<<nblocks, kBlkThreads, 0, s>>>(probs, blk, coef, launch);
    else k_batch_blocked<4><<<nblocks, kBlkThreads, 0, s>>>(probs, blk, coef, launch);
    return hipGetLastError();
}

hipError_t launch_batch_convert(BatchProbDev* probs, const int* ids, const int* blk_start, int nseg, int nblocks,
                                int to_fp32, hipStream_t s) {
    if (nseg == 0 || nblocks == 0) return hipSuccess;
    k_batch_convert<<<nblocks, 256, 0, s>>>(probs, ids, blk_start, nseg, to_fp32);
    return hipGetLastError();
}

hipError_t launch_batch_mgs(const BatchMgsDev* info, const MgsLink* links, int nprob, const int* blk_start,
                            int nblocks, int ell, double* partial, double* hout, hipStream_t s) {
    k_batch_mgs<<<nblocks, 256, 0, s>>>(info, links, nprob, blk_start, ell, partial, hout);
    return hipGetLastError();
}

}  // namespace ew
