// Initial guess by projection on earlier solves (P. F. Fischer, "Projection
// techniques for iterative solution of Ax = b with successive right-hand
// sides", CMAME 163, 1998).  The operator keeps the last proj_k solutions x_k
// (M x_k = b_k) in FP32, across wave-solves.  For a new right-hand side b the
// guess x0 = sum_k alpha_k x_k minimises the M-norm of the error x* - x0 over
// their span; the normal equations are
//   sum_j (x_i . M x_j) alpha_j = x_i . b,   x_i . M x_j = x_i . b_j = x_j . b_i,
// so only products of stored solutions with right-hand sides are needed.  The
// products x_k . b computed for the guess are, by the symmetry of M, the new
// row of the Gram matrix G[i][j] = x_i . b_j once x is solved; only the
// diagonal x . b is added after the solve, and the b_k need not be kept.
#include <cmath>

#include "dense.h"
#include "op.h"
#include "stencil_dev.h"

namespace ew {
namespace {

struct ProjArgs {
    int k;                    // active slots 0..k-1
    double alpha[kProjMax];   // combination weights
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Reduce acc[0..kProjMax] over the block; block b writes partial[v * kProjBlocks + b].
__device__ __forceinline__ void block_store(double (&acc)[kProjMax + 1], int nv, double* __restrict__ partial) {
    __shared__ double red[4][kProjMax + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v <= kProjMax; ++v) {
        if (v < nv || v == kProjMax) {
            const double s = wave_sum(acc[v]);
            if (lane == 0) red[wave][v] = s;
        }
    }
    __syncthreads();
    const int v = threadIdx.x;
    if (v <= kProjMax && (v < nv || v == kProjMax))
        partial[(int64_t)v * kProjBlocks + blockIdx.x] = (red[0][v] + red[1][v]) + (red[2][v] + red[3][v]);
}

// Stored solutions are rows of X with leading dimension ld (a multiple of 4,
// zero beyond N), read four points at a time.
__device__ __forceinline__ void load_b4(const double* __restrict__ b, int64_t i, int64_t N, double (&bv)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) bv[e] = (i + e < N) ? b[i + e] : 0.0;
}

// partial sets: v < k: x_v . b;  v = kProjMax: b . b
__global__ __launch_bounds__(256) void k_proj_dots(const float* __restrict__ X, int64_t N, int64_t ld, ProjArgs pa,
                                                   const double* __restrict__ b, double* __restrict__ partial) {
    double acc[kProjMax + 1];
#pragma unroll
    for (int v = 0; v <= kProjMax; ++v) acc[v] = 0.0;
    const int64_t nq = (N + 3) / 4;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nq; q += (int64_t)kProjBlocks * 256) {
        const int64_t i = 4 * q;
        double bv[4];
        load_b4(b, i, N, bv);
#pragma unroll
        for (int v = 0; v < kProjMax; ++v) {
            if (v < pa.k) {
                const float4 xv = *reinterpret_cast<const float4*>(X + (int64_t)v * ld + i);
                acc[v] += ((double)xv.x * bv[0] + (double)xv.y * bv[1]) + ((double)xv.z * bv[2] + (double)xv.w * bv[3]);
            }
        }
        acc[kProjMax] += (bv[0] * bv[0] + bv[1] * bv[1]) + (bv[2] * bv[2] + bv[3] * bv[3]);
    }
    block_store(acc, pa.k, partial);
}

// X[new] = x; partial kProjMax: x . (bscale b).
__global__ __launch_bounds__(256) void k_proj_add(float* __restrict__ X, int64_t N, int64_t ld, int newslot,
                                                  const double* __restrict__ x, const double* __restrict__ b,
                                                  double bscale, double* __restrict__ partial) {
    double acc[kProjMax + 1];
#pragma unroll
    for (int v = 0; v <= kProjMax; ++v) acc[v] = 0.0;
    float* xn = X + (int64_t)newslot * ld;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kProjBlocks * 256) {
        const double xi = x[i];
        xn[i] = (float)xi;
        acc[kProjMax] += xi * (bscale * b[i]);
    }
    block_store(acc, 0, partial);
}

// out[v] = sum over blocks of partial[v][.]; one workgroup per value v
// (blockIdx.x < k, or the last one for v = kProjMax), fixed order.
__global__ __launch_bounds__(256) void k_proj_finish(const double* __restrict__ partial, int k,
                                                     double* __restrict__ out) {
    const int v = (int)blockIdx.x < k ? (int)blockIdx.x : kProjMax;
    double s = 0.0;
    for (int b = threadIdx.x; b < kProjBlocks; b += 256) s += partial[(int64_t)v * kProjBlocks + b];
    const double t = block_sum_256(s, threadIdx.x);
    if (threadIdx.x == 0) out[v] = t;
}

__global__ __launch_bounds__(256) void k_proj_combine(const float* __restrict__ X, int64_t N, int64_t ld, ProjArgs pa,
                                                      double* __restrict__ x0) {
    const int64_t nq = (N + 3) / 4;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nq; q += (int64_t)gridDim.x * 256) {
        const int64_t i = 4 * q;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int v = 0; v < kProjMax; ++v) {
            if (v < pa.k) {
                const float4 xv = *reinterpret_cast<const float4*>(X + (int64_t)v * ld + i);
                const double al = pa.alpha[v];
                s0 += al * (double)xv.x;
                s1 += al * (double)xv.y;
                s2 += al * (double)xv.z;
                s3 += al * (double)xv.w;
            }
        }
        if (i < N) x0[i] = s0;
        if (i + 1 < N) x0[i + 1] = s1;
        if (i + 2 < N) x0[i + 2] = s2;
        if (i + 3 < N) x0[i + 3] = s3;
    }
}

}  // namespace

ew_status Op::proj_setup() {
    const bool wants = implicit && (desc.predictor == EW_PRED_PROJ || desc.predictor == EW_PRED_CNN);
    const int k = desc.proj_window == 0 ? 24 : desc.proj_window;
    if (!wants || k <= 0) return EW_OK;
    proj_k = k;
    proj_ld = (N + 63) / 64 * 64;
    EW_TRY(alloc((void**)&proj_X, (size_t)k * proj_ld * sizeof(float)));
    // the padding beyond N is read (times zero) by the four-point kernels: clear it once
    EW_HIP_TRY(hipMemset(proj_X, 0, (size_t)k * proj_ld * sizeof(float)));
    EW_TRY(alloc((void**)&proj_partial, 2 * (size_t)kProjBlocks * (kProjMax + 1) * sizeof(double)));
    EW_TRY(alloc((void**)&proj_res_dev, 2 * (kProjMax + 1) * sizeof(double)));
    EW_HIP_TRY(hipHostMalloc((void**)&proj_res_host, 2 * (kProjMax + 1) * sizeof(double), hipHostMallocDefault));
    proj_G.assign((size_t)kProjMax * kProjMax, 0.0);
    proj_c.assign(kProjMax, 0.0);
    return EW_OK;
}

// x <- the projection guess for M x = bscale b (zero while nothing is stored).
ew_status Op::proj_guess(const double* b, double bscale, double* x, bool* x_is_zero) {
    *x_is_zero = true;
    proj_rhs_ok = false;
    if (proj_k <= 0) return EW_OK;
    if (proj_count == 0) {
        proj_rhs_ok = true;  // nothing to combine; the first pair starts the window
        return EW_OK;
    }
    ProjArgs pa{};
    pa.k = proj_count;
    k_proj_dots<<<kProjBlocks, 256, 0, stream>>>(proj_X, N, proj_ld, pa, b, proj_partial);
    EW_HIP_TRY(hipGetLastError());
    k_proj_finish<<<proj_count + 1, 256, 0, stream>>>(proj_partial, proj_count, proj_res_dev);
    EW_HIP_TRY(hipGetLastError());
    // one copy brings the products with b and, if pending, the last pair's Gram row
    EW_HIP_TRY(hipMemcpyAsync(proj_res_host, proj_res_dev, 2 * (kProjMax + 1) * sizeof(double),
                              hipMemcpyDeviceToHost, stream));
    EW_HIP_TRY(hipStreamSynchronize(stream));
    const double* c = proj_res_host;
    if (proj_pending) {
        proj_G[(size_t)proj_pending_slot * kProjMax + proj_pending_slot] = proj_res_host[(kProjMax + 1) + kProjMax];
        proj_pending = false;
    }
    const double bb = c[kProjMax];
    if (!std::isfinite(bb)) return fail(EW_ERR_NONFINITE, "non-finite right-hand side");
    bb_src = b;
    bb_val = bb;
    if (bb == 0.0) return EW_OK;
    for (int v = 0; v < proj_count; ++v) proj_c[v] = bscale * c[v];  // x_v . (bscale b): the next Gram row
    proj_rhs_ok = true;
    // Normal equations with unit diagonal, solved by a Cholesky factorisation
    // that admits the stored pairs newest first and skips a pair whose pivot
    // falls below kDrop (to that level it is a combination of the pairs
    // already admitted).  A ridge instead of the skip would damp the
    // small-eigenvalue directions that carry most of the guess's accuracy.
    constexpr double kDrop = 1e-10;
    const int k = proj_count;
    std::vector<double> d(k);
    for (int v = 0; v < k; ++v) {
        const double gv = proj_G[(size_t)v * kProjMax + v];
        if (!(gv > 0.0) || !std::isfinite(gv)) return EW_OK;  // degenerate history: fall back to zero
        d[v] = 1.0 / std::sqrt(gv);
    }
    auto A = [&](int i, int j) { return d[i] * proj_G[(size_t)i * kProjMax + j] * d[j]; };
    std::vector<int> idx;               // admitted slots, in factor order
    Mat Lc(k, k);                       // lower factor of A[idx][idx]
    for (int a = 0; a < k; ++a) {
        const int j = ((proj_head - 1 - a) % proj_k + proj_k) % proj_k;  // newest first
        const int m = (int)idx.size();
        std::vector<double> l(m);
        double piv = A(j, j);
        for (int r = 0; r < m; ++r) {
            double t = A(idx[r], j);
            for (int q = 0; q < r; ++q) t -= Lc(r, q) * l[q];
            l[r] = t / Lc(r, r);
            piv -= l[r] * l[r];
        }
        if (!(piv > kDrop)) continue;
        for (int r = 0; r < m; ++r) Lc(m, r) = l[r];
        Lc(m, m) = std::sqrt(piv);
        idx.push_back(j);
    }
    const int m = (int)idx.size();
    std::vector<double> y(m);
    for (int i = 0; i < m; ++i) {
        double t = proj_c[idx[i]] * d[idx[i]];
        for (int q = 0; q < i; ++q) t -= Lc(i, q) * y[q];
        y[i] = t / Lc(i, i);
    }
    for (int i = m - 1; i >= 0; --i) {
        double t = y[i];
        for (int q = i + 1; q < m; ++q) t -= Lc(q, i) * y[q];
        y[i] = t / Lc(i, i);
    }
    for (int v = 0; v < kProjMax; ++v) pa.alpha[v] = 0.0;
    for (int i = 0; i < m; ++i) pa.alpha[idx[i]] = d[idx[i]] * y[i];
    const int64_t blocks = std::min<int64_t>(((N + 3) / 4 + 255) / 256, 2048);
    k_proj_combine<<<(unsigned)blocks, 256, 0, stream>>>(proj_X, N, proj_ld, pa, x);
    EW_HIP_TRY(hipGetLastError());
    *x_is_zero = false;
    proj_guesses++;
    return EW_OK;
}

// Store the solution x of M x = bscale b in the ring: its Gram row against the
// other stored solutions is proj_c (computed for the guess); the diagonal
// x . (bscale b) follows on the device and is read with the next guess.
ew_status Op::proj_add(const double* b, double bscale, const double* x) {
    if (proj_k <= 0 || !proj_rhs_ok) return EW_OK;
    const int slot = proj_head;
    const int prev_count = proj_count;
    proj_head = (proj_head + 1) % proj_k;
    if (proj_count < proj_k) ++proj_count;
    for (int v = 0; v < prev_count; ++v) {
        if (v == slot) continue;  // the pair being replaced
        proj_G[(size_t)slot * kProjMax + v] = proj_c[v];
        proj_G[(size_t)v * kProjMax + slot] = proj_c[v];
    }
    double* part = proj_partial + (size_t)kProjBlocks * (kProjMax + 1);
    k_proj_add<<<kProjBlocks, 256, 0, stream>>>(proj_X, N, proj_ld, slot, x, b, bscale, part);
    EW_HIP_TRY(hipGetLastError());
    k_proj_finish<<<1, 256, 0, stream>>>(part, 0, proj_res_dev + (kProjMax + 1));
    EW_HIP_TRY(hipGetLastError());
    proj_pending = true;
    proj_pending_slot = slot;
    proj_rhs_ok = false;
    return EW_OK;
}

}  // namespace ew
