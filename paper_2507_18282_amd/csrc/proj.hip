// Initial guess by projection on earlier solves (P. F. Fischer, "Projection
// techniques for iterative solution of Ax = b with successive right-hand
// sides", CMAME 163, 1998).  The operator keeps the last proj_k pairs
// (x_k, b_k) with M x_k = b_k in FP32, across wave-solves.  For a new
// right-hand side b the guess x0 = sum_k alpha_k x_k minimises the M-norm of
// the error x* - x0 over their span; the normal equations are
//   sum_j (x_i . M x_j) alpha_j = x_i . b,   with x_i . M x_j = x_i . b_j,
// so only inner products with stored vectors are needed.  The Gram matrix
// G[i][j] = x_i . b_j lives on the host and gains one row per solve.
#include <cmath>

#include "dense.h"
#include "op.h"
#include "stencil_dev.h"

namespace ew {
namespace {

struct ProjArgs {
    int k;                    // active slots 0..k-1
    int newslot;              // slot written by the add kernel
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

// partial sets: v < k: x_v . b;  v = kProjMax: b . b
__global__ __launch_bounds__(256) void k_proj_dots(const float* __restrict__ X, int64_t N, ProjArgs pa,
                                                   const double* __restrict__ b, double* __restrict__ partial) {
    double acc[kProjMax + 1];
#pragma unroll
    for (int v = 0; v <= kProjMax; ++v) acc[v] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kProjBlocks * 256) {
        const double bi = b[i];
#pragma unroll
        for (int v = 0; v < kProjMax; ++v)
            if (v < pa.k) acc[v] += (double)X[(int64_t)v * N + i] * bi;
        acc[kProjMax] += bi * bi;
    }
    block_store(acc, pa.k, partial);
}

// X[new] = x, B[new] = bscale b; partial v < k: x . b_v (the new b in FP64 for v = new).
__global__ __launch_bounds__(256) void k_proj_add(float* __restrict__ X, float* __restrict__ B, int64_t N,
                                                  ProjArgs pa, const double* __restrict__ x,
                                                  const double* __restrict__ b, double bscale,
                                                  double* __restrict__ partial) {
    double acc[kProjMax + 1];
#pragma unroll
    for (int v = 0; v <= kProjMax; ++v) acc[v] = 0.0;
    const int64_t no = (int64_t)pa.newslot * N;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kProjBlocks * 256) {
        const double xi = x[i];
        const double bi = bscale * b[i];
        X[no + i] = (float)xi;
        B[no + i] = (float)bi;
#pragma unroll
        for (int v = 0; v < kProjMax; ++v)
            if (v < pa.k) acc[v] += xi * (v == pa.newslot ? bi : (double)B[(int64_t)v * N + i]);
    }
    block_store(acc, pa.k, partial);
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

__global__ __launch_bounds__(256) void k_proj_combine(const float* __restrict__ X, int64_t N, ProjArgs pa,
                                                      double* __restrict__ x0) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < kProjMax; ++v)
            if (v < pa.k) s += pa.alpha[v] * (double)X[(int64_t)v * N + i];
        x0[i] = s;
    }
}

}  // namespace

ew_status Op::proj_setup() {
    const bool wants = implicit && (desc.predictor == EW_PRED_PROJ || desc.predictor == EW_PRED_CNN);
    const int k = desc.proj_window == 0 ? 24 : desc.proj_window;
    if (!wants || k <= 0) return EW_OK;
    proj_k = k;
    EW_TRY(alloc((void**)&proj_X, (size_t)k * N * sizeof(float)));
    EW_TRY(alloc((void**)&proj_B, (size_t)k * N * sizeof(float)));
    EW_TRY(alloc((void**)&proj_partial, 2 * (size_t)kProjBlocks * (kProjMax + 1) * sizeof(double)));
    EW_TRY(alloc((void**)&proj_res_dev, 2 * (kProjMax + 1) * sizeof(double)));
    EW_HIP_TRY(hipHostMalloc((void**)&proj_res_host, 2 * (kProjMax + 1) * sizeof(double), hipHostMallocDefault));
    proj_G.assign((size_t)kProjMax * kProjMax, 0.0);
    return EW_OK;
}

// x <- the projection guess for M x = bscale b (zero while nothing is stored).
ew_status Op::proj_guess(const double* b, double bscale, double* x, bool* x_is_zero) {
    *x_is_zero = true;
    if (proj_k <= 0 || proj_count == 0) return EW_OK;
    ProjArgs pa{};
    pa.k = proj_count;
    pa.newslot = -1;
    k_proj_dots<<<kProjBlocks, 256, 0, stream>>>(proj_X, N, pa, b, proj_partial);
    EW_HIP_TRY(hipGetLastError());
    k_proj_finish<<<proj_count + 1, 256, 0, stream>>>(proj_partial, proj_count, proj_res_dev);
    EW_HIP_TRY(hipGetLastError());
    // one copy brings the products with b and, if pending, the last pair's Gram row
    EW_HIP_TRY(hipMemcpyAsync(proj_res_host, proj_res_dev, 2 * (kProjMax + 1) * sizeof(double),
                              hipMemcpyDeviceToHost, stream));
    EW_HIP_TRY(hipStreamSynchronize(stream));
    const double* c = proj_res_host;
    if (proj_pending) {
        const double* g = proj_res_host + (kProjMax + 1);
        const int s = proj_pending_slot;
        for (int v = 0; v < proj_count; ++v) {
            proj_G[(size_t)s * kProjMax + v] = g[v];
            proj_G[(size_t)v * kProjMax + s] = g[v];
        }
        proj_pending = false;
    }
    const double bb = c[kProjMax];
    if (!std::isfinite(bb)) return fail(EW_ERR_NONFINITE, "non-finite right-hand side");
    bb_src = b;
    bb_val = bb;
    if (bb == 0.0) return EW_OK;
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
        double t = bscale * c[idx[i]] * d[idx[i]];
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
    const int64_t blocks = std::min<int64_t>((N + 255) / 256, 2048);
    k_proj_combine<<<(unsigned)blocks, 256, 0, stream>>>(proj_X, N, pa, x);
    EW_HIP_TRY(hipGetLastError());
    *x_is_zero = false;
    proj_guesses++;
    return EW_OK;
}

// Store the solved pair (x, bscale b) in the ring and start its Gram row.
ew_status Op::proj_add(const double* b, double bscale, const double* x) {
    if (proj_k <= 0) return EW_OK;
    const int slot = proj_head;
    proj_head = (proj_head + 1) % proj_k;
    if (proj_count < proj_k) ++proj_count;
    ProjArgs pa{};
    pa.k = proj_count;
    pa.newslot = slot;
    double* part = proj_partial + (size_t)kProjBlocks * (kProjMax + 1);
    k_proj_add<<<kProjBlocks, 256, 0, stream>>>(proj_X, proj_B, N, pa, x, b, bscale, part);
    EW_HIP_TRY(hipGetLastError());
    k_proj_finish<<<proj_count + 1, 256, 0, stream>>>(part, proj_count, proj_res_dev + (kProjMax + 1));
    EW_HIP_TRY(hipGetLastError());
    proj_pending = true;
    proj_pending_slot = slot;
    return EW_OK;
}

}  // namespace ew
