// FP64 vector kernels of the Arnoldi process: deterministic reductions, the
// chained modified Gram-Schmidt links, tall-skinny basis rotations and Gram
// blocks, and the SplitMix64 start-vector generator.
//
// These are HBM-bound GEMV/GEMM shapes (arithmetic intensity <= k/8 flop/B for
// k <= 64 columns, far below the FP64 ridge), so they use vector FMA; every
// reduction runs over a fixed grid of kRedBlocks blocks with a fixed order of
// additions, so repeated runs are bitwise identical.
#include "stencil_dev.h"

namespace ew {

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                     int64_t n, double* __restrict__ partial) {
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)kRedBlocks * 256)
        acc += x[c] * y[c];
    const double s = block_sum_256(acc, threadIdx.x);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* partial, hipStream_t s) {
    k_dot_partial<<<kRedBlocks, 256, 0, s>>>(x, y, n, partial);
    return hipGetLastError();
}

// One link of the modified Gram-Schmidt chain (Alg. "Arnoldi"): the previous
// kernel left the partial sums of h = (w, v_prev); finish that sum, subtract
// h v_prev from w, and start the next inner product (w, v_next) in the same
// pass.  Each link reads w, v_prev, v_next and writes w.
// With vnext == w the new inner product is the squared norm of the updated w.
__global__ __launch_bounds__(256) void k_mgs_link(double* w, const double* __restrict__ vprev, const double* vnext,
                                                  int64_t n, const double* __restrict__ partial_in,
                                                  double* __restrict__ partial_out, double* __restrict__ h_out) {
    const double h = sum_partials(partial_in);
    if (blockIdx.x == 0 && threadIdx.x == 0 && h_out) *h_out = h;
    const bool self = (vnext == w);
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)kRedBlocks * 256) {
        const double wi = w[c] - h * vprev[c];
        w[c] = wi;
        acc += wi * (self ? wi : vnext[c]);
    }
    const double s = block_sum_256(acc, threadIdx.x);
    if (threadIdx.x == 0) partial_out[blockIdx.x] = s;
}

hipError_t launch_mgs_link(double* w, const double* vprev, const double* vnext, int64_t n, const double* partial_in,
                           double* partial_out, double* h_out, hipStream_t s) {
    k_mgs_link<<<kRedBlocks, 256, 0, s>>>(w, vprev, vnext, n, partial_in, partial_out, h_out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_normalize(const double* __restrict__ w, double* __restrict__ v, int64_t n,
                                                   const double* __restrict__ partial_in, double* __restrict__ nrm_out) {
    const double nrm = sqrt(sum_partials(partial_in));
    if (blockIdx.x == 0 && threadIdx.x == 0 && nrm_out) *nrm_out = nrm;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)kRedBlocks * 256)
        v[c] = w[c] / nrm;
}

hipError_t launch_normalize_from_partial(const double* w, double* v, int64_t n, const double* partial_in,
                                         double* nrm_out, hipStream_t s) {
    k_normalize<<<kRedBlocks, 256, 0, s>>>(w, v, n, partial_in, nrm_out);
    return hipGetLastError();
}

// Y[:, c] = V[:, 0:nv] Q[0:nv, c] for a chunk of up to 16 output columns per
// launch pass; each thread owns one row, and Q passes through LDS in slabs of
// kGemmSlab rows (any nv).
constexpr int kGemmCols = 16;
constexpr int kGemmSlab = 320;

__global__ __launch_bounds__(256) void k_tall_gemm(const double* __restrict__ V, int64_t n, int nv,
                                                   const double* __restrict__ Q, int ldq, int c0, int nc,
                                                   double* __restrict__ Y) {
    __shared__ double q[kGemmSlab * kGemmCols];
    for (int64_t rb = (int64_t)blockIdx.x * 256; rb < n; rb += (int64_t)gridDim.x * 256) {
        const int64_t r = rb + threadIdx.x;
        double acc[kGemmCols];
#pragma unroll
        for (int c = 0; c < kGemmCols; ++c) acc[c] = 0.0;
        for (int i0 = 0; i0 < nv; i0 += kGemmSlab) {
            const int ni = (nv - i0) < kGemmSlab ? (nv - i0) : kGemmSlab;
            __syncthreads();
            for (int t = threadIdx.x; t < ni * nc; t += 256) {
                const int i = t % ni, c = t / ni;
                q[i * kGemmCols + c] = Q[(i0 + i) + (int64_t)(c0 + c) * ldq];
            }
            __syncthreads();
            if (r < n) {
                for (int i = 0; i < ni; ++i) {
                    const double vi = V[(int64_t)(i0 + i) * n + r];
#pragma unroll
                    for (int c = 0; c < kGemmCols; ++c) acc[c] += vi * q[i * kGemmCols + c];
                }
            }
        }
        if (r < n) {
#pragma unroll
            for (int c = 0; c < kGemmCols; ++c)
                if (c < nc) Y[(int64_t)(c0 + c) * n + r] = acc[c];
        }
    }
}

hipError_t launch_tall_gemm(const double* V, int64_t n, int nv, const double* Q_dev, int ldq, int ncols, double* Y,
                            hipStream_t s) {
    if (nv < 1 || ncols < 1) return hipErrorInvalidValue;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    for (int c0 = 0; c0 < ncols; c0 += kGemmCols) {
        const int nc = (ncols - c0) < kGemmCols ? (ncols - c0) : kGemmCols;
        k_tall_gemm<<<(unsigned)blocks, 256, 0, s>>>(V, n, nv, Q_dev, ldq, c0, nc, Y);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block classical Gram-Schmidt over a basis of many columns (the columns of
// two column-major blocks, [U1 | U2], leading dimension n): h = U^T w by
// row-slice partials, then w -= U h.  Twice applied this is CGS2, whose
// orthogonality matches MGS's while every pass streams the basis once with
// full parallelism instead of one launch per column.
// ---------------------------------------------------------------------------
struct ColPair {
    const double* u1;
    int n1;
    const double* u2;
};

__device__ __forceinline__ const double* col_at(const ColPair& U, int c, int64_t n) {
    return c < U.n1 ? U.u1 + (int64_t)c * n : U.u2 + (int64_t)(c - U.n1) * n;
}

// partial[s * nu + c] = sum over rows of slice s of U[:, c] * w; one wavefront
// per (column, slice), four columns per workgroup.
__global__ __launch_bounds__(256) void k_block_dot(ColPair U, int nu, const double* __restrict__ w, int64_t n,
                                                   int64_t slice, double* __restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nu) return;
    const int64_t r0 = (int64_t)blockIdx.y * slice;
    int64_t r1 = r0 + slice;
    if (r1 > n) r1 = n;
    const double* u = col_at(U, c, n);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t r = r0 + lane;
    for (; r + 192 < r1; r += 256) {
        a0 += u[r] * w[r];
        a1 += u[r + 64] * w[r + 64];
        a2 += u[r + 128] * w[r + 128];
        a3 += u[r + 192] * w[r + 192];
    }
    for (; r < r1; r += 64) a0 += u[r] * w[r];
    double v = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) partial[(int64_t)blockIdx.y * nu + c] = v;
}

// h_cur[c] = sum_s partial[s * nu + c] (slices in order); h_tot[c] = h_cur[c]
// on the first pass, += on the second.
__global__ __launch_bounds__(256) void k_block_dot_sum(const double* __restrict__ partial, int nslices, int nu,
                                                       double* __restrict__ h_cur, double* __restrict__ h_tot,
                                                       int accumulate) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= nu) return;
    double v = 0.0;
    for (int s = 0; s < nslices; ++s) v += partial[(int64_t)s * nu + c];
    h_cur[c] = v;
    h_tot[c] = accumulate ? h_tot[c] + v : v;
}

// Columns [k * chunk, (k+1) * chunk) of U times h for the rows of this block
// (h passes through LDS in slabs of kAxpySlab): with one chunk, w -= U h
// directly; else the chunk's product goes to tmp[k * n + r] for
// k_block_axpy_sum.
constexpr int kAxpySlab = 512;
__global__ __launch_bounds__(256) void k_block_axpy(ColPair U, int nu, const double* __restrict__ h, int chunk,
                                                    double* __restrict__ w, int64_t n, double* __restrict__ tmp) {
    __shared__ double hs[kAxpySlab];
    const int c0 = blockIdx.y * chunk;
    int c1 = c0 + chunk;
    if (c1 > nu) c1 = nu;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = r < n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int s0 = c0; s0 < c1; s0 += kAxpySlab) {
        const int ns = (c1 - s0) < kAxpySlab ? (c1 - s0) : kAxpySlab;
        __syncthreads();
        for (int t = threadIdx.x; t < ns; t += 256) hs[t] = h[s0 + t];
        __syncthreads();
        if (live) {
            int c = 0;
            for (; c + 3 < ns; c += 4) {
                a0 += col_at(U, s0 + c, n)[r] * hs[c];
                a1 += col_at(U, s0 + c + 1, n)[r] * hs[c + 1];
                a2 += col_at(U, s0 + c + 2, n)[r] * hs[c + 2];
                a3 += col_at(U, s0 + c + 3, n)[r] * hs[c + 3];
            }
            for (; c < ns; ++c) a0 += col_at(U, s0 + c, n)[r] * hs[c];
        }
    }
    if (!live) return;
    const double acc = (a0 + a1) + (a2 + a3);
    if (gridDim.y == 1)
        w[r] -= acc;
    else
        tmp[(int64_t)blockIdx.y * n + r] = acc;
}

__global__ __launch_bounds__(256) void k_block_axpy_sum(const double* __restrict__ tmp, int nchunks,
                                                        double* __restrict__ w, int64_t n) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double v = 0.0;
    for (int k = 0; k < nchunks; ++k) v += tmp[(int64_t)k * n + r];
    w[r] -= v;
}

// ---------------------------------------------------------------------------
// Modified Gram-Schmidt of one short vector (n <= kMgsSmallMax) in a single
// workgroup: w stays in registers (PTS points per thread), each basis column
// is read once (its next column is loaded while the current inner product is
// reduced), and every inner product is a fixed-order workgroup reduction, so
// results are repeatable.  h_out[0:nu] receives the coefficients and h_out[nu]
// the norm before normalisation; w is overwritten by w / ||w||.  Replaces the
// chain of nu + 2 launches that latency dominates on grids of a few thousand
// points.
// ---------------------------------------------------------------------------
constexpr int kMgsSmallThreads = 1024;

__device__ __forceinline__ double wg_sum_1024(double v, double* red) {
    // red: 16 doubles of this round's buffer; every thread gets the same total
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += red[i];
    return t;
}

template <int PTS>
__global__ __launch_bounds__(kMgsSmallThreads) void k_mgs_small(ColPair U, int nu, double* __restrict__ w, int n,
                                                                double* __restrict__ h_out) {
    __shared__ double red[2][16];
    const int tid = threadIdx.x;
    double wr[PTS], ua[PTS], ub[PTS];
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        const int q = tid + t * kMgsSmallThreads;
        wr[t] = q < n ? w[q] : 0.0;
    }
    if (nu > 0) {
        const double* u0 = col_at(U, 0, n);
#pragma unroll
        for (int t = 0; t < PTS; ++t) {
            const int q = tid + t * kMgsSmallThreads;
            ua[t] = q < n ? u0[q] : 0.0;
        }
    }
    for (int c = 0; c < nu; ++c) {
        // prefetch the next column
        if (c + 1 < nu) {
            const double* un = col_at(U, c + 1, n);
#pragma unroll
            for (int t = 0; t < PTS; ++t) {
                const int q = tid + t * kMgsSmallThreads;
                ub[t] = q < n ? un[q] : 0.0;
            }
        }
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < PTS; ++t) part += wr[t] * ua[t];
        const double h = wg_sum_1024(part, red[c & 1]);
#pragma unroll
        for (int t = 0; t < PTS; ++t) wr[t] -= h * ua[t];
        if (tid == 0) h_out[c] = h;
#pragma unroll
        for (int t = 0; t < PTS; ++t) ua[t] = ub[t];
    }
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < PTS; ++t) part += wr[t] * wr[t];
    const double nrm = sqrt(wg_sum_1024(part, red[nu & 1]));
    if (tid == 0) h_out[nu] = nrm;
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        const int q = tid + t * kMgsSmallThreads;
        if (q < n) w[q] = wr[t] / nrm;
    }
}

hipError_t launch_mgs_small(const double* u1, int n1, const double* u2, int n2, double* w, int64_t n, double* h_out,
                            hipStream_t s) {
    if (n < 1 || n > kMgsSmallMax || n1 < 0 || n2 < 0) return hipErrorInvalidValue;
    const ColPair U{u1, n1, u2};
    const int nu = n1 + n2, ni = (int)n;
    if (n <= 4 * kMgsSmallThreads)
        k_mgs_small<4><<<1, kMgsSmallThreads, 0, s>>>(U, nu, w, ni, h_out);
    else
        k_mgs_small<8><<<1, kMgsSmallThreads, 0, s>>>(U, nu, w, ni, h_out);
    return hipGetLastError();
}

BlockGsPlan block_gs_plan(int64_t n, int nu) {
    BlockGsPlan p{};
    // dot: at least 4096 wavefronts where the slices stay >= 1024 rows
    int64_t ns = (4096 + nu - 1) / nu;
    const int64_t ns_max = (n + 1023) / 1024;
    if (ns > ns_max) ns = ns_max;
    if (ns > kBlockGsMaxSlices) ns = kBlockGsMaxSlices;
    if (ns < 1) ns = 1;
    p.slice = (n + ns - 1) / ns;
    p.nslices = (int)((n + p.slice - 1) / p.slice);
    // axpy: split the columns when there are fewer than 2048 row blocks
    const int64_t rb = (n + 255) / 256;
    int64_t nc = (2048 + rb - 1) / rb;
    const int64_t nc_cols = (nu + 15) / 16;
    if (nc > nc_cols) nc = nc_cols;
    if (nc > kBlockGsMaxChunks) nc = kBlockGsMaxChunks;
    if (nc < 1) nc = 1;
    const int64_t chunk = (nu + nc - 1) / nc;
    p.chunk = (int)chunk;
    p.nchunks = (int)((nu + chunk - 1) / chunk);
    return p;
}

hipError_t launch_block_gs_pass(const double* u1, int n1, const double* u2, int n2, double* w, int64_t n,
                                const BlockGsPlan& p, double* partial, double* h_cur, double* h_tot, int accumulate,
                                double* tmp, hipStream_t s) {
    const int nu = n1 + n2;
    if (nu < 1) return hipErrorInvalidValue;
    if (p.nchunks > 1 && (int64_t)p.nchunks * n > kBlockGsTmpDoubles) return hipErrorInvalidValue;
    const ColPair U{u1, n1, u2};
    k_block_dot<<<dim3((unsigned)((nu + 3) / 4), (unsigned)p.nslices), 256, 0, s>>>(U, nu, w, n, p.slice, partial);
    k_block_dot_sum<<<(nu + 255) / 256, 256, 0, s>>>(partial, p.nslices, nu, h_cur, h_tot, accumulate);
    const unsigned rb = (unsigned)((n + 255) / 256);
    k_block_axpy<<<dim3(rb, (unsigned)p.nchunks), 256, 0, s>>>(U, nu, h_cur, p.chunk, w, n, tmp);
    if (p.nchunks > 1) k_block_axpy_sum<<<rb, 256, 0, s>>>(tmp, p.nchunks, w, n);
    return hipGetLastError();
}

// Gram block partials: block b accumulates sum_r A[r, i] B[r, j] over its
// contiguous range of rows for i < na, j < nb (na, nb <= 32), staging 32 rows
// of both blocks through LDS at a time.
constexpr int kGramMax = 32;
__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ A, int na, const double* __restrict__ B,
                                                      int nb, int64_t n, double* __restrict__ partial) {
    __shared__ double ta[32][kGramMax + 1];
    __shared__ double tb[32][kGramMax + 1];
    const int np = na * nb;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // pairs tid, tid+256, tid+512, tid+768
    const int64_t rows_per_block = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    for (int64_t r0 = r_begin; r0 < r_end; r0 += 32) {
        for (int t = threadIdx.x; t < 32 * na; t += 256) {
            const int rr = t % 32, c = t / 32;
            const int64_t r = r0 + rr;
            ta[rr][c] = (r < r_end) ? A[(int64_t)c * n + r] : 0.0;
        }
        for (int t = threadIdx.x; t < 32 * nb; t += 256) {
            const int rr = t % 32, c = t / 32;
            const int64_t r = r0 + rr;
            tb[rr][c] = (r < r_end) ? B[(int64_t)c * n + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = threadIdx.x + 256 * q;
            if (p < np) {
                const int i = p / nb, j = p % nb;
                double s = 0.0;
                for (int rr = 0; rr < 32; ++rr) s += ta[rr][i] * tb[rr][j];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int p = threadIdx.x + 256 * q;
        if (p < np) partial[(int64_t)blockIdx.x * np + p] = acc[q];
    }
}

hipError_t launch_gram_partial(const double* A, int na, const double* B, int nb, int64_t n, double* partial,
                               int nblocks, hipStream_t s) {
    if (na > kGramMax || nb > kGramMax || na < 1 || nb < 1) return hipErrorInvalidValue;
    k_gram_partial<<<nblocks, 256, 0, s>>>(A, na, B, nb, n, partial);
    return hipGetLastError();
}

// Partials of ||lz + mu z||^2 (first kRedBlocks entries) and ||z||^2 (next kRedBlocks).
__global__ __launch_bounds__(256) void k_eig_residual(const double* __restrict__ lz, const double* __restrict__ z,
                                                      double mu, int64_t n, double* __restrict__ partial) {
    double a0 = 0.0, a1 = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)kRedBlocks * 256) {
        const double r = lz[c] + mu * z[c];
        a0 += r * r;
        a1 += z[c] * z[c];
    }
    const double s0 = block_sum_256(a0, threadIdx.x);
    if (threadIdx.x == 0) partial[blockIdx.x] = s0;
    const double s1 = block_sum_256(a1, threadIdx.x);
    if (threadIdx.x == 0) partial[kRedBlocks + blockIdx.x] = s1;
}

hipError_t launch_eig_residual(const double* lz, const double* z, double mu, int64_t n, double* partial,
                               hipStream_t s) {
    k_eig_residual<<<kRedBlocks, 256, 0, s>>>(lz, z, mu, n, partial);
    return hipGetLastError();
}

// Per block: the entry of largest magnitude (the first such index) of y;
// partial[b] = its value, partial[kRedBlocks + b] = its index (exact in FP64),
// -1 for a block that sees no entry.
__global__ __launch_bounds__(256) void k_absmax_partial(const double* __restrict__ y, int64_t n,
                                                        double* __restrict__ partial) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double bv = 0.0;
    int64_t bi = -1;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)kRedBlocks * 256) {
        const double v = y[c];
        if (bi < 0 || fabs(v) > fabs(bv)) {  // indices grow along the scan, so ties keep the first
            bv = v;
            bi = c;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double ov = sv[threadIdx.x + off];
            const int64_t oi = si[threadIdx.x + off];
            const double mv = sv[threadIdx.x];
            const int64_t mi = si[threadIdx.x];
            const bool take = oi >= 0 && (mi < 0 || fabs(ov) > fabs(mv) || (fabs(ov) == fabs(mv) && oi < mi));
            if (take) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = sv[0];
        partial[kRedBlocks + blockIdx.x] = (double)si[0];
    }
}

hipError_t launch_absmax_partial(const double* y, int64_t n, double* partial, hipStream_t s) {
    k_absmax_partial<<<kRedBlocks, 256, 0, s>>>(y, n, partial);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea, Flood 2014; Vigna's finaliser constants), counter
// form: z_i = mix(seed + (i+1) * golden); value = 2 * (z_i >> 11) * 2^-53 - 1.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_splitmix_uniform(double* __restrict__ x, int64_t n, uint64_t seed) {
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
        const uint64_t z = splitmix_at(seed, (uint64_t)c);
        x[c] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    }
}

hipError_t launch_splitmix_uniform(double* x, int64_t n, uint64_t seed, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_splitmix_uniform<<<(unsigned)blocks, 256, 0, s>>>(x, n, seed);
    return hipGetLastError();
}

}  // namespace ew
