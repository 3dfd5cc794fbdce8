// A single curvilinear grid by the mapping method (Sec. "Discrete
// approximations"): the order-2 Laplacian in conservative form,
//
//   J L_h u = D+r (A11 D-r u) + D+s (A22 D-s u) + D0r (B D0s u) + D0s (B D0r u),
//
// J = x_r y_s - x_s y_r, J a^11 = (x_s^2 + y_s^2)/J, J a^22 = (x_r^2 + y_r^2)/J,
// B = J a^12 = -(x_r x_s + y_r y_s)/J, A11 (A22) at a half point the mean of
// J a^11 (J a^22) at its two nodes, metric derivatives by centred differences
// of the grid coordinates, Dirichlet walls (u = 0).  J L_h is symmetric, so
// L_h is self-adjoint in the inner product weighted by J; the eigensolver
// works in y = J^{1/2} u.
//
// The coefficients are built once on the host from the caller's coordinates
// and kept on the device as four arrays (A11 / dr^2 at x half points, A22 /
// ds^2 at y half points, B / (4 dr ds) and 1/J at the nodes).  The explicit
// steps run several per launch in LDS-staged tiles (mapped_steps.hip).  The
// implicit scheme solves M = I - (dt^2/2) L_h by multigrid whose coarse
// levels carry the Galerkin product R M P of the level above as nine
// weights per point (on a non-orthogonal grid it contracts the error about
// twice as fast per cycle as rediscretising J a^{mn} on the coarse points),
// with zebra line
// relaxation along the first parameter direction (point red-black
// Gauss-Seidel on levels whose lines exceed the LDS), full weighting and
// bilinear prolongation.
#include <cmath>
#include <memory>
#include <vector>

#include "op.h"
#include "stencil_dev.h"

namespace ew {

// L_h u at active point (i, j), c = j nx + i; values beyond the walls are 0.
// A cross term whose node lies on a wall multiplies a difference of wall
// values, so it is dropped rather than read.
__device__ __forceinline__ double lap_mapped(const double* __restrict__ u, int64_t c, int i, int j, const Geo& g,
                                             const MapCoef& m) {
    const int nx = g.nx;
    const bool w = i > 0, e = i < nx - 1, s = j > 0, n = j < g.ny - 1;
    const double uc = u[c];
    const double uW = w ? u[c - 1] : 0.0, uE = e ? u[c + 1] : 0.0;
    const double uS = s ? u[c - nx] : 0.0, uN = n ? u[c + nx] : 0.0;
    const double uSW = (w && s) ? u[c - nx - 1] : 0.0, uSE = (e && s) ? u[c - nx + 1] : 0.0;
    const double uNW = (w && n) ? u[c + nx - 1] : 0.0, uNE = (e && n) ? u[c + nx + 1] : 0.0;
    const int64_t hw = (int64_t)j * (nx + 1) + i;  // half point i - 1/2
    double t = m.cw[hw + 1] * (uE - uc) - m.cw[hw] * (uc - uW);
    t += m.cs[c + nx] * (uN - uc) - m.cs[c] * (uc - uS);
    const double bE = e ? m.cb[c + 1] : 0.0, bW = w ? m.cb[c - 1] : 0.0;
    const double bN = n ? m.cb[c + nx] : 0.0, bS = s ? m.cb[c - nx] : 0.0;
    t += bE * (uNE - uSE) - bW * (uNW - uSW);  // D0r (B D0s u)
    t += bN * (uNE - uNW) - bS * (uSE - uSW);  // D0s (B D0r u)
    return m.ij[c] * t;
}

__global__ __launch_bounds__(256) void k_laplacian_mapped(const double* __restrict__ u, double* __restrict__ out,
                                                          Geo g, MapCoef m) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, 0);
    out[c] = lap_mapped(u, c, i, j, g, m);
}

__global__ __launch_bounds__(256) void k_pointwise_mul(const double* in, const double* __restrict__ f, double* out,
                                                       int64_t n) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        out[c] = in[c] * f[c];
}

hipError_t launch_laplacian_mapped(const double* u, double* out, const Geo& g, const MapCoef& m, hipStream_t s) {
    k_laplacian_mapped<<<tile_grid(g), dim3(kTileX, kTileY, 1), 0, s>>>(u, out, g, m);
    return hipGetLastError();
}

hipError_t launch_pointwise_mul(const double* in, const double* f, double* out, int64_t n, hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    k_pointwise_mul<<<(unsigned)b, 256, 0, s>>>(in, f, out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Multigrid on mapped levels (implicit scheme): M = I - a L_h from the
// coefficients on the finest level, from nine Galerkin weights per point on
// the coarser ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mdiag_mapped(int64_t c, int i, int j, const Geo& g, const MapCoef& m, double a) {
    const int64_t hw = (int64_t)j * (g.nx + 1) + i;
    const double centre = -(m.cw[hw + 1] + m.cw[hw] + m.cs[c + g.nx] + m.cs[c]);
    return 1.0 - a * m.ij[c] * centre;
}

// (M x)_c from the nine weights of a Galerkin level; values beyond the walls are 0
__device__ __forceinline__ double apply_gw(const double* __restrict__ x, int64_t c, int i, int j, const Geo& g,
                                           const double* __restrict__ gw) {
    const int nx = g.nx;
    const int64_t n = g.size();
    const bool w = i > 0, e = i < nx - 1, s = j > 0, nn = j < g.ny - 1;
    double t = gw[c] * x[c];
    if (w) t += gw[n + c] * x[c - 1];
    if (e) t += gw[2 * n + c] * x[c + 1];
    if (s) {
        t += gw[3 * n + c] * x[c - nx];
        if (w) t += gw[5 * n + c] * x[c - nx - 1];
        if (e) t += gw[6 * n + c] * x[c - nx + 1];
    }
    if (nn) {
        t += gw[4 * n + c] * x[c + nx];
        if (w) t += gw[7 * n + c] * x[c + nx - 1];
        if (e) t += gw[8 * n + c] * x[c + nx + 1];
    }
    return t;
}

// residual b_c - (M x)_c of a mapped level (GEN: Galerkin weights)
template <bool GEN>
__device__ __forceinline__ double resid_at(const double* __restrict__ x, const double* __restrict__ b, double bscale,
                                           int64_t c, int i, int j, const Geo& g, const MapCoef& m, double a) {
    if (GEN) return bscale * b[c] - apply_gw(x, c, i, j, g, m.gw);
    return bscale * b[c] - (x[c] - a * lap_mapped(x, c, i, j, g, m));
}

template <bool GEN>
__global__ __launch_bounds__(256) void k_rb_half_mapped(const double* __restrict__ xin, double* __restrict__ xout,
                                                        const double* __restrict__ b, double bscale, Geo g, MapCoef m,
                                                        double a, double w, int colour) {
    int i, j, k;
    if (!tile_coords(g, i, j, k)) return;
    const int64_t c = lin(g, i, j, 0);
    const double xc = xin[c];
    if (((i + j) & 1) != colour) {
        xout[c] = xc;
        return;
    }
    const double r = resid_at<GEN>(xin, b, bscale, c, i, j, g, m, a);
    xout[c] = xc + w * r / (GEN ? m.gw[c] : mdiag_mapped(c, i, j, g, m, a));
}

template <bool GEN>
__global__ __launch_bounds__(256) void k_residual_mapped(const double* __restrict__ x, const double* __restrict__ b,
                                                         double bscale, Geo g, MapCoef m, double a,
                                                         double* __restrict__ partial, double* __restrict__ r_out) {
    const int64_t n = g.size();
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
        const int i = (int)(c % g.nx), j = (int)(c / g.nx);
        const double r = resid_at<GEN>(x, b, bscale, c, i, j, g, m, a);
        if (r_out) r_out[c] = r;
        acc += r * r;
    }
    if (partial) {  // uniform over the block
        const double s = block_sum_256(acc, threadIdx.x);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// Full weighting: coarse point (I, J) sits on fine point (2I + 1, 2J + 1);
// weights 1/4, 1/2, 1/4 per direction (n_f = 2 n_c + 1, so every fine index
// read is in range).
__global__ __launch_bounds__(256) void k_restrict_fw(const double* __restrict__ r, Geo gf, double* __restrict__ bc,
                                                     Geo gc) {
    int I, J, k;
    if (!tile_coords(gc, I, J, k)) return;
    const int fi = 2 * I + 1, fj = 2 * J + 1;
    double sum = 0.0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
        const double* row = r + (int64_t)(fj + dj) * gf.nx + fi;
        const double v = 0.25 * row[-1] + 0.5 * row[0] + 0.25 * row[1];
        sum += (dj == 0 ? 0.5 : 0.25) * v;
    }
    bc[lin(gc, I, J, 0)] = sum;
}

hipError_t launch_rb_half_mapped(const double* xin, double* xout, const double* b, double bscale, const Geo& g,
                                 const MapCoef& m, double a, double w, int colour, hipStream_t s) {
    const dim3 grid = tile_grid(g), block(kTileX, kTileY, 1);
    if (m.gw) k_rb_half_mapped<true><<<grid, block, 0, s>>>(xin, xout, b, bscale, g, m, a, w, colour);
    else k_rb_half_mapped<false><<<grid, block, 0, s>>>(xin, xout, b, bscale, g, m, a, w, colour);
    return hipGetLastError();
}

hipError_t launch_residual_mapped(const double* x, const double* b, double bscale, const Geo& g, const MapCoef& m,
                                  double a, double* partial, double* r_out, hipStream_t s) {
    if (m.gw) k_residual_mapped<true><<<kRedBlocks, 256, 0, s>>>(x, b, bscale, g, m, a, partial, r_out);
    else k_residual_mapped<false><<<kRedBlocks, 256, 0, s>>>(x, b, bscale, g, m, a, partial, r_out);
    return hipGetLastError();
}

hipError_t launch_restrict_fw(const double* r, const Geo& gf, double* bc, const Geo& gc, hipStream_t s) {
    k_restrict_fw<<<tile_grid(gc), dim3(kTileX, kTileY, 1), 0, s>>>(r, gf, bc, gc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Zebra line relaxation.  On a mapped grid the coupling along one parameter
// direction can be several times the coupling along the other (the cells of
// an annulus sector are elongated in the angle), and point Gauss-Seidel stops
// smoothing the error that varies slowly along the strong direction; relaxing
// whole grid lines removes it.  One workgroup owns one line j of the parity
// being relaxed.  It forms the line's right-hand side b_i + a/J (couplings to
// lines j - 1 and j + 1, which no other workgroup of the launch writes) with
// coalesced reads and solves the tridiagonal system with the Thomas factors
// made on the host: the forward and backward substitutions are first-order
// linear recurrences, each evaluated as a scan of affine maps y -> A + B y
// over the 256 threads (one contiguous segment of the line per thread).
// The line lives in LDS, padded by one slot per segment so that the threads'
// strided segment reads fall in distinct banks; the super-diagonal factors
// wait in registers until the forward pass has used the sub-diagonal ones,
// and then take their slots, so a line needs two arrays of LDS.
// ---------------------------------------------------------------------------
constexpr int kLineThreads = 256;

__device__ __forceinline__ int line_seg(int nx) { return (nx + kLineThreads - 1) / kLineThreads; }

// points a thread stages per line (lines of up to kLineStage * kLineThreads points)
constexpr int kLineStage = 12;

// two line arrays in 48 KB of LDS (nx <= 2816; with the scan's wave totals,
// three workgroups fit in one CU's LDS)
bool line_relax_fits(int nx) {
    return nx >= 1 && nx <= kLineStage * kLineThreads && 2 * (size_t)(nx + kLineThreads) * sizeof(double) <= 49152;
}

// (A, B) <- (A, B) o (A2, B2): the map that applies (A2, B2) first
__device__ __forceinline__ void compose_after(double& A, double& B, double A2, double B2) {
    A = A + B * A2;
    B = B * B2;
}

// Inclusive scan of affine maps over the block; FORWARD: thread t gets
// f_t o ... o f_0, else f_t o ... o f_255.  Returns, through `in`, the value
// entering the thread's segment when the recurrence starts from 0 (the first
// component of the composition of all segments before it).
template <bool FORWARD>
__device__ __forceinline__ double scan_entry(double A, double B, double* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double Ao = FORWARD ? __shfl_up(A, off, 64) : __shfl_down(A, off, 64);
        const double Bo = FORWARD ? __shfl_up(B, off, 64) : __shfl_down(B, off, 64);
        if (FORWARD ? lane >= off : lane + off < 64) compose_after(A, B, Ao, Bo);
    }
    if (lane == (FORWARD ? 63 : 0)) {
        wsum[2 * w] = A;
        wsum[2 * w + 1] = B;
    }
    __syncthreads();
    // composition of the other waves' totals that precede this wave in the
    // direction of the recurrence
    double PA = 0.0, PB = 1.0;
    if (FORWARD) {
        for (int v = 0; v < w; ++v) {
            double TA = wsum[2 * v], TB = wsum[2 * v + 1];
            compose_after(TA, TB, PA, PB);
            PA = TA;
            PB = TB;
        }
    } else {
        for (int v = kLineThreads / 64 - 1; v > w; --v) {
            double TA = wsum[2 * v], TB = wsum[2 * v + 1];
            compose_after(TA, TB, PA, PB);
            PA = TA;
            PB = TB;
        }
    }
    compose_after(A, B, PA, 0.0);  // only the first component is needed below
    const double nb = FORWARD ? __shfl_up(A, 1, 64) : __shfl_down(A, 1, 64);
    __syncthreads();  // wsum is reused by the next scan
    return (FORWARD ? lane == 0 : lane == 63) ? PA : nb;
}

template <bool GEN>
__global__ __launch_bounds__(kLineThreads) void k_line_half_mapped(double* x, const double* __restrict__ b,
                                                                   double bscale, Geo g, MapCoef m, double a,
                                                                   double w, int parity) {
    extern __shared__ double lds[];
    __shared__ double wsum[2 * (kLineThreads / 64)];
    const int nx = g.nx, ny = g.ny;
    const int j = parity + 2 * (int)blockIdx.x;
    if (j >= ny) return;  // uniform per block
    const int S = line_seg(nx);
    const int np = nx + kLineThreads;
    double* P = lds;       // alpha -> y -> x
    double* Q = lds + np;  // tl, then tu
    const int64_t row = (int64_t)j * nx;
    const bool has_s = j > 0, has_n = j < ny - 1;
    double tur[kLineStage];  // tu of the staged points, stored once tl is used up
#pragma unroll
    for (int k = 0; k < kLineStage; ++k) {
        const int i = (int)threadIdx.x + k * kLineThreads;
        if (i >= nx) break;
        const int64_t c = row + i;
        const bool w = i > 0, e = i < nx - 1;
        double rhs;
        if (GEN) {
            // b minus the couplings to lines j - 1 and j + 1
            const int64_t n = (int64_t)nx * ny;
            const double* gw = m.gw;
            double t = 0.0;
            if (has_s) {
                const double* xs = x + c - nx;
                t += gw[3 * n + c] * xs[0];
                if (w) t += gw[5 * n + c] * xs[-1];
                if (e) t += gw[6 * n + c] * xs[1];
            }
            if (has_n) {
                const double* xn = x + c + nx;
                t += gw[4 * n + c] * xn[0];
                if (w) t += gw[7 * n + c] * xn[-1];
                if (e) t += gw[8 * n + c] * xn[1];
            }
            rhs = bscale * b[c] - t;
        } else {
            double t = 0.0;
            if (has_s) {
                const double* xs = x + c - nx;
                const double uS = xs[0], uSW = w ? xs[-1] : 0.0, uSE = e ? xs[1] : 0.0;
                t += m.cs[c] * uS - m.cb[c - nx] * (uSE - uSW);
                const double bE = e ? m.cb[c + 1] : 0.0, bW = w ? m.cb[c - 1] : 0.0;
                t += bW * uSW - bE * uSE;
            }
            if (has_n) {
                const double* xn = x + c + nx;
                const double uN = xn[0], uNW = w ? xn[-1] : 0.0, uNE = e ? xn[1] : 0.0;
                t += m.cs[c + nx] * uN + m.cb[c + nx] * (uNE - uNW);
                const double bE = e ? m.cb[c + 1] : 0.0, bW = w ? m.cb[c - 1] : 0.0;
                t += bE * uNE - bW * uNW;
            }
            rhs = bscale * b[c] + a * m.ij[c] * t;
        }
        const int p = i + i / S;
        P[p] = rhs * m.tw[c];
        Q[p] = m.tl[c];
        tur[k] = m.tu[c];
    }
    __syncthreads();
    const int lo = threadIdx.x * S, hi = min(lo + S, nx);
    const int pb = lo + (int)threadIdx.x;  // padded position of lo (lo / S = thread index)
    // forward substitution y_i = alpha_i - tl_i y_{i-1}, y_{-1} = 0
    double A = 0.0, B = 1.0;
    for (int i = lo; i < hi; ++i) {
        const int p = pb + (i - lo);
        double gA = P[p], gB = -Q[p];
        compose_after(gA, gB, A, B);
        A = gA;
        B = gB;
    }
    double y = scan_entry<true>(A, B, wsum);
    for (int i = lo; i < hi; ++i) {
        const int p = pb + (i - lo);
        y = P[p] - Q[p] * y;
        P[p] = y;
    }
    __syncthreads();  // every tl read: the slots take tu
#pragma unroll
    for (int k = 0; k < kLineStage; ++k) {
        const int i = (int)threadIdx.x + k * kLineThreads;
        if (i >= nx) break;
        Q[i + i / S] = tur[k];
    }
    __syncthreads();
    // backward substitution x_i = y_i - tu_i x_{i+1}, x_nx = 0
    A = 0.0;
    B = 1.0;
    for (int i = hi - 1; i >= lo; --i) {
        const int p = pb + (i - lo);
        double gA = P[p], gB = -Q[p];
        compose_after(gA, gB, A, B);
        A = gA;
        B = gB;
    }
    double xv = scan_entry<false>(A, B, wsum);
    for (int i = hi - 1; i >= lo; --i) {
        const int p = pb + (i - lo);
        xv = P[p] - Q[p] * xv;
        P[p] = xv;
    }
    __syncthreads();
    // the line's solution, or with a weight w != 1 the over-relaxed update
    // x + w (solution - x) (successive line over-relaxation); line j is
    // written by this workgroup only
    if (w == 1.0) {
        for (int i = threadIdx.x; i < nx; i += kLineThreads) x[row + i] = P[i + i / S];
    } else {
        for (int i = threadIdx.x; i < nx; i += kLineThreads) {
            const double old = x[row + i];
            x[row + i] = old + w * (P[i + i / S] - old);
        }
    }
}

hipError_t launch_line_half_mapped(double* x, const double* b, double bscale, const Geo& g, const MapCoef& m,
                                   double a, double w, int parity, hipStream_t s) {
    if (!line_relax_fits(g.nx) || !m.tw || (parity != 0 && parity != 1)) return hipErrorInvalidValue;
    const int lines = (g.ny - parity + 1) / 2;
    if (lines <= 0) return hipSuccess;
    const size_t lds = 2 * (size_t)(g.nx + kLineThreads) * sizeof(double);
    if (m.gw) k_line_half_mapped<true><<<lines, kLineThreads, lds, s>>>(x, b, bscale, g, m, a, w, parity);
    else k_line_half_mapped<false><<<lines, kLineThreads, lds, s>>>(x, b, bscale, g, m, a, w, parity);
    return hipGetLastError();
}

// V(nu1, nu2) cycle on mapped level l from the iterate in cur (zero if
// `zero`); other is its partner buffer and holds the residual while the
// coarser levels run.  A full sweep is a red half-sweep into other and a
// black one back, so the result is always in cur.
ew_status Op::mapped_vcycle(int l, double* cur, double* other, const double* b, double bscale, bool zero,
                            double** result) {
    const Level& L = levels[l];
    const MapCoef& m = mcoef[l];
    const int64_t n = L.g.size();
    const double w = level_relax(l);  // 1 on a level of one point (an exact solve)
    auto sweeps = [&](int count, bool from_zero) -> ew_status {
        if (from_zero) EW_HIP_TRY(launch_fill<double>(cur, n, 0.0, stream));
        for (int s = 0; s < count; ++s) {
            if (m.tw) {
                // per relaxed point: x on the two neighbouring lines, b, 1/J, two
                // A22 and three B values, three factors; write x (and read the
                // line's old x when over-relaxed)
                ProfScope ps(this, EW_K_SMOOTH, l, (w == 1.0 ? 104.0 : 112.0) * (double)n);
                EW_HIP_TRY(launch_line_half_mapped(cur, b, bscale, L.g, m, a, w, 0, stream));
                EW_HIP_TRY(launch_line_half_mapped(cur, b, bscale, L.g, m, a, w, 1, stream));
            } else {
                ProfScope ps(this, EW_K_SMOOTH, l, 48.0 * (double)n);
                EW_HIP_TRY(launch_rb_half_mapped(cur, other, b, bscale, L.g, m, a, w, 0, stream));
                EW_HIP_TRY(launch_rb_half_mapped(other, cur, b, bscale, L.g, m, a, w, 1, stream));
            }
        }
        return EW_OK;
    };
    *result = cur;
    if (l == (int)levels.size() - 1) return sweeps(n == 1 ? 1 : desc.mg_coarse_sweeps, zero);
    EW_TRY(sweeps(desc.mg_nu1, zero));
    const Level& C = levels[l + 1];
    {
        ProfScope ps(this, EW_K_RESTRICT, l, 8.0 * (3.0 * (double)n + (double)C.g.size()));
        EW_HIP_TRY(launch_residual_mapped(cur, b, bscale, L.g, m, a, nullptr, other, stream));
        EW_HIP_TRY(launch_restrict_fw(other, L.g, (double*)C.b, C.g, stream));
    }
    double* xc = nullptr;
    EW_TRY(mapped_vcycle(l + 1, (double*)C.x[0], (double*)C.x[1], (const double*)C.b, 1.0, true, &xc));
    {
        ProfScope ps(this, EW_K_PROLONG, l, 8.0 * (2.0 * (double)n + (double)C.g.size()));
        EW_HIP_TRY(launch_prolong_correct<double>(cur, xc, L.g, C.g, stream));
    }
    return sweeps(desc.mg_nu2, false);
}

// ---------------------------------------------------------------------------
// Host: coefficients from the coordinates.  xy holds x then y, each
// (n1 + 4) x (n2 + 4) with node (i, j), i in [-2, n1 + 1], at (i + 2) +
// (n1 + 4)(j + 2); metric terms are formed at the nodes i in [-1, n1],
// j in [-1, n2] (walls included).  A coarse multigrid level with spacing
// 2^l dr samples them at its own nodes, which are fine nodes.
// ---------------------------------------------------------------------------
namespace {

struct Nodes {
    int n1 = 0, n2 = 0;
    std::vector<double> J, a11, a22, a12;  // (n1 + 2) x (n2 + 2), node (i, j) at (i + 1) + (n1 + 2)(j + 1)
};

struct HostCoef {
    std::vector<double> cw, cs, cb, ij, sq, isq;
    double rho = 0.0;    // Gershgorin bound on the spectrum of -L_h
    double rho_j = 0.0;  // Gershgorin ratio of M = I - a L_h: off-diagonal row sum over diagonal
};

ew_status node_metrics(const double* xy, int n1, int n2, Nodes& nd) {
    const int64_t px = n1 + 4, plane = px * (int64_t)(n2 + 4);
    for (int64_t q = 0; q < 2 * plane; ++q)
        if (!std::isfinite(xy[q])) return fail(EW_ERR_INVALID_ARG, "mapped grid coordinates must be finite");
    const double dr = 1.0 / (n1 + 1), ds = 1.0 / (n2 + 1);
    auto X = [&](int i, int j) { return xy[(i + 2) + px * (j + 2)]; };
    auto Y = [&](int i, int j) { return xy[plane + (i + 2) + px * (j + 2)]; };
    const int64_t nx2 = n1 + 2, ny2 = n2 + 2;
    nd.n1 = n1;
    nd.n2 = n2;
    nd.J.assign(nx2 * ny2, 0.0);
    nd.a11.assign(nx2 * ny2, 0.0);
    nd.a22.assign(nx2 * ny2, 0.0);
    nd.a12.assign(nx2 * ny2, 0.0);
    for (int j = -1; j <= n2; ++j)
        for (int i = -1; i <= n1; ++i) {
            const double xr = (X(i + 1, j) - X(i - 1, j)) / (2.0 * dr), yr = (Y(i + 1, j) - Y(i - 1, j)) / (2.0 * dr);
            const double xs = (X(i, j + 1) - X(i, j - 1)) / (2.0 * ds), ys = (Y(i, j + 1) - Y(i, j - 1)) / (2.0 * ds);
            const double jac = xr * ys - xs * yr;
            if (!(jac > 0.0) || !std::isfinite(jac))
                return fail(EW_ERR_INVALID_ARG, "mapped grid: the Jacobian x_r y_s - x_s y_r must be positive at every "
                                                "node (walls included)");
            const int64_t q = (i + 1) + nx2 * (j + 1);
            nd.J[q] = jac;
            nd.a11[q] = (xs * xs + ys * ys) / jac;
            nd.a22[q] = (xr * xr + yr * yr) / jac;
            nd.a12[q] = -(xr * xs + yr * ys) / jac;
        }
    return EW_OK;
}

// Coefficients of the level with nl1 x nl2 points whose node (I, J) is fine
// node (stride (I + 1) - 1, stride (J + 1) - 1); a is the implicit weight (0
// when only rho is wanted).
void level_coefficients(const Nodes& nd, int stride, int nl1, int nl2, double a, HostCoef& hc) {
    const int64_t nx2 = nd.n1 + 2;
    auto at = [&](const std::vector<double>& F, int I, int J) {
        const int i = stride * (I + 1) - 1, j = stride * (J + 1) - 1;
        return F[(i + 1) + nx2 * (j + 1)];
    };
    const double dr = stride / (double)(nd.n1 + 1), ds = stride / (double)(nd.n2 + 1);
    const int64_t N = (int64_t)nl1 * nl2;
    hc.cw.assign((int64_t)(nl1 + 1) * nl2, 0.0);
    hc.cs.assign((int64_t)nl1 * (nl2 + 1), 0.0);
    hc.cb.assign(N, 0.0);
    hc.ij.assign(N, 0.0);
    hc.sq.assign(N, 0.0);
    hc.isq.assign(N, 0.0);
    const double idr2 = 1.0 / (dr * dr), ids2 = 1.0 / (ds * ds), q4 = 1.0 / (4.0 * dr * ds);
    for (int j = 0; j < nl2; ++j)
        for (int hi = 0; hi <= nl1; ++hi)
            hc.cw[hi + (int64_t)(nl1 + 1) * j] = 0.5 * (at(nd.a11, hi - 1, j) + at(nd.a11, hi, j)) * idr2;
    for (int hj = 0; hj <= nl2; ++hj)
        for (int i = 0; i < nl1; ++i)
            hc.cs[i + (int64_t)nl1 * hj] = 0.5 * (at(nd.a22, i, hj - 1) + at(nd.a22, i, hj)) * ids2;
    double rho = 0.0, rho_j = 0.0;
    for (int j = 0; j < nl2; ++j)
        for (int i = 0; i < nl1; ++i) {
            const int64_t c = i + (int64_t)nl1 * j;
            const double jac = at(nd.J, i, j);
            hc.cb[c] = at(nd.a12, i, j) * q4;
            hc.ij[c] = 1.0 / jac;
            hc.sq[c] = std::sqrt(jac);
            hc.isq[c] = 1.0 / hc.sq[c];
            // Gershgorin: (1/J) times the absolute sum of the nine weights of
            // J L_h, the cross weights of wall nodes included
            const double wE = hc.cw[(i + 1) + (int64_t)(nl1 + 1) * j], wW = hc.cw[i + (int64_t)(nl1 + 1) * j];
            const double wN = hc.cs[i + (int64_t)nl1 * (j + 1)], wS = hc.cs[c];
            const double bE = at(nd.a12, i + 1, j) * q4, bW = at(nd.a12, i - 1, j) * q4;
            const double bN = at(nd.a12, i, j + 1) * q4, bS = at(nd.a12, i, j - 1) * q4;
            const double centre = std::fabs(wE + wW + wN + wS);
            const double off = std::fabs(wE) + std::fabs(wW) + std::fabs(wN) + std::fabs(wS) + std::fabs(bE + bN) +
                               std::fabs(bE + bS) + std::fabs(bW + bN) + std::fabs(bW + bS);
            rho = std::max(rho, (centre + off) / jac);
            rho_j = std::max(rho_j, a * off / jac / (1.0 + a * centre / jac));
        }
    hc.rho = rho;
    hc.rho_j = rho_j;
}

ew_status upload(Op* op, const std::vector<double>& h, const double** dst) {
    double* d = nullptr;
    EW_TRY(op->alloc((void**)&d, h.size() * sizeof(double)));
    EW_HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    *dst = d;
    return EW_OK;
}

// Thomas factors of the line systems of M = I - a L_h on one level: along
// line j, d_i x_i + l_i x_{i-1} + u_i x_{i+1} = rhs_i with d_i the diagonal
// of M and l_i, u_i its couplings to the points beside i on the line (the
// diagonally dominant rows need no pivoting).
void line_factors(const HostCoef& hc, int nl1, int nl2, double a, std::vector<double>& tw, std::vector<double>& tl,
                  std::vector<double>& tu) {
    const int64_t N = (int64_t)nl1 * nl2;
    tw.assign(N, 0.0);
    tl.assign(N, 0.0);
    tu.assign(N, 0.0);
    for (int j = 0; j < nl2; ++j) {
        double cp = 0.0;
        for (int i = 0; i < nl1; ++i) {
            const int64_t c = i + (int64_t)nl1 * j, hw = i + (int64_t)(nl1 + 1) * j;
            const double s = a * hc.ij[c];
            const double d = 1.0 + s * (hc.cw[hw] + hc.cw[hw + 1] + hc.cs[c] + hc.cs[c + nl1]);
            const double l = i > 0 ? -s * hc.cw[hw] : 0.0;
            const double u = i < nl1 - 1 ? -s * hc.cw[hw + 1] : 0.0;
            const double w = 1.0 / (d - l * cp);
            tw[c] = w;
            tl[c] = l * w;
            tu[c] = cp = u * w;
        }
    }
}

// M = I - a L_h of one level as nine weights per point, w[k N + c] for the
// offsets k = C, W, E, S, N, SW, SE, NW, NE (weights to points beyond a
// wall are 0).
constexpr int kDx[9] = {0, -1, 1, 0, 0, -1, 1, -1, 1};
constexpr int kDy[9] = {0, 0, 0, -1, 1, -1, -1, 1, 1};

struct Stencil9 {
    int nx = 0, ny = 0;
    std::vector<double> w;
};

int stencil_slot(int dx, int dy) {
    for (int k = 0; k < 9; ++k)
        if (kDx[k] == dx && kDy[k] == dy) return k;
    return -1;
}

// The finest level's weights from its coefficients (the operator of lap_mapped).
void fine_stencil(const HostCoef& hc, int nx, int ny, double a, Stencil9& st) {
    const int64_t N = (int64_t)nx * ny;
    st.nx = nx;
    st.ny = ny;
    st.w.assign(9 * N, 0.0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int64_t c = i + (int64_t)nx * j, hw = i + (int64_t)(nx + 1) * j;
            const bool w = i > 0, e = i < nx - 1, s = j > 0, n = j < ny - 1;
            const double f = -a * hc.ij[c];
            const double cwW = hc.cw[hw], cwE = hc.cw[hw + 1], csS = hc.cs[c], csN = hc.cs[c + nx];
            const double bE = e ? hc.cb[c + 1] : 0.0, bW = w ? hc.cb[c - 1] : 0.0;
            const double bN = n ? hc.cb[c + nx] : 0.0, bS = s ? hc.cb[c - nx] : 0.0;
            double* W = st.w.data() + c;
            W[0] = 1.0 - f * (cwW + cwE + csS + csN);
            if (w) W[1 * N] = f * cwW;
            if (e) W[2 * N] = f * cwE;
            if (s) W[3 * N] = f * csS;
            if (n) W[4 * N] = f * csN;
            if (s && w) W[5 * N] = f * (bW + bS);
            if (s && e) W[6 * N] = -f * (bE + bS);
            if (n && w) W[7 * N] = -f * (bW + bN);
            if (n && e) W[8 * N] = f * (bE + bN);
        }
}

// Galerkin coarse operator R M P: P bilinear interpolation from coarse node
// (I, J) = fine node (2I + 1, 2J + 1), R = P^T / 4 (full weighting).
void galerkin(const Stencil9& F, Stencil9& C) {
    const int nfx = F.nx, nfy = F.ny, ncx = (nfx - 1) / 2, ncy = (nfy - 1) / 2;
    const int64_t NF = (int64_t)nfx * nfy, NC = (int64_t)ncx * ncy;
    C.nx = ncx;
    C.ny = ncy;
    C.w.assign(9 * NC, 0.0);
    // coarse nodes whose hat covers fine index f (0-based) and the hat's value
    auto cover = [](int f, int nc, int* idx, double* wt) -> int {
        if (f & 1) {
            idx[0] = (f - 1) / 2;
            wt[0] = 1.0;
            return (idx[0] >= 0 && idx[0] < nc) ? 1 : 0;
        }
        int cnt = 0;
        for (int q : {f / 2 - 1, f / 2})
            if (q >= 0 && q < nc) {
                idx[cnt] = q;
                wt[cnt++] = 0.5;
            }
        return cnt;
    };
    for (int J = 0; J < ncy; ++J)
        for (int I = 0; I < ncx; ++I) {
            double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int ry = -1; ry <= 1; ++ry)
                for (int rx = -1; rx <= 1; ++rx) {
                    const int fx = 2 * I + 1 + rx, fy = 2 * J + 1 + ry;
                    const double rw = (rx == 0 ? 0.5 : 0.25) * (ry == 0 ? 0.5 : 0.25);
                    const int64_t f = fx + (int64_t)nfx * fy;
                    for (int k = 0; k < 9; ++k) {
                        const int gx = fx + kDx[k], gy = fy + kDy[k];
                        if (gx < 0 || gx >= nfx || gy < 0 || gy >= nfy) continue;
                        const double wv = F.w[k * NF + f];
                        if (wv == 0.0) continue;
                        int ix[2], iy[2];
                        double px[2], py[2];
                        const int cx = cover(gx, ncx, ix, px), cy = cover(gy, ncy, iy, py);
                        for (int u = 0; u < cx; ++u)
                            for (int v = 0; v < cy; ++v) {
                                const int slot = stencil_slot(ix[u] - I, iy[v] - J);
                                if (slot >= 0) acc[slot] += rw * wv * px[u] * py[v];
                            }
                    }
                }
            const int64_t c = I + (int64_t)ncx * J;
            for (int k = 0; k < 9; ++k) C.w[k * NC + c] = acc[k];
        }
}

// Gershgorin ratio of a stencil's rows: off-diagonal absolute sum over the diagonal.
double stencil_rho_j(const Stencil9& st) {
    const int64_t N = (int64_t)st.nx * st.ny;
    double r = 0.0;
    for (int64_t c = 0; c < N; ++c) {
        double off = 0.0;
        for (int k = 1; k < 9; ++k) off += std::fabs(st.w[k * N + c]);
        r = std::max(r, off / std::fabs(st.w[c]));
    }
    return r;
}

// Thomas factors of the line systems (W, C, E weights) of a stencil, as line_factors.
void stencil_line_factors(const Stencil9& st, std::vector<double>& tw, std::vector<double>& tl,
                          std::vector<double>& tu) {
    const int64_t N = (int64_t)st.nx * st.ny;
    tw.assign(N, 0.0);
    tl.assign(N, 0.0);
    tu.assign(N, 0.0);
    for (int j = 0; j < st.ny; ++j) {
        double cp = 0.0;
        for (int i = 0; i < st.nx; ++i) {
            const int64_t c = i + (int64_t)st.nx * j;
            const double d = st.w[c];
            const double l = i > 0 ? st.w[N + c] : 0.0;
            const double u = i < st.nx - 1 ? st.w[2 * N + c] : 0.0;
            const double w = 1.0 / (d - l * cp);
            tw[c] = w;
            tl[c] = l * w;
            tu[c] = cp = u * w;
        }
    }
}

ew_status upload_level(Op* op, const HostCoef& hc, MapCoef& m) {
    EW_TRY(upload(op, hc.cw, &m.cw));
    EW_TRY(upload(op, hc.cs, &m.cs));
    EW_TRY(upload(op, hc.cb, &m.cb));
    EW_TRY(upload(op, hc.ij, &m.ij));
    EW_TRY(upload(op, hc.sq, &m.sq));
    EW_TRY(upload(op, hc.isq, &m.isq));
    return EW_OK;
}

// Levels halve (n - 1)/2 while both sizes are odd and >= 3, up to
// mg_max_levels; with EW_MG_LEVELS_AUTO the hierarchy stops at the first
// level whose Gauss-Seidel contraction bound rho_J^2, raised to
// mg_coarse_sweeps, is at most 0.1 (rho_J from that level's operator).
// Coarse levels carry the Galerkin product R M P of the level above.
ew_status build_mapped_hierarchy(Op* op, const Nodes& nd, const HostCoef& fine) {
    const ew_op_desc& d = op->desc;
    const size_t max_levels = d.mg_max_levels > 0 ? (size_t)d.mg_max_levels : 64;
    int nl1 = nd.n1, nl2 = nd.n2, stride = 1;
    Stencil9 st;  // the current level's operator (coarse levels: Galerkin products)
    fine_stencil(fine, nl1, nl2, op->a, st);
    for (;;) {
        Level L;
        const int64_t nn[3] = {nl1, nl2, 1};
        const double hh[3] = {stride / (double)(nd.n1 + 1), stride / (double)(nd.n2 + 1), 1.0};
        L.g = make_geo(2, nn, hh, 0);
        const int64_t n = L.g.size();
        MapCoef m{};
        std::vector<double> tw, tl, tu;
        if (stride == 1) {
            m = op->mc;
            EW_TRY(op->alloc(&L.x[1], n * sizeof(double)));
            if (line_relax_fits(nl1)) line_factors(fine, nl1, nl2, op->a, tw, tl, tu);
        } else {
            EW_TRY(upload(op, st.w, &m.gw));
            EW_TRY(op->alloc(&L.x[0], n * sizeof(double)));
            EW_TRY(op->alloc(&L.x[1], n * sizeof(double)));
            EW_TRY(op->alloc(&L.b, n * sizeof(double)));
            if (line_relax_fits(nl1)) stencil_line_factors(st, tw, tl, tu);
        }
        if (!tw.empty()) {
            EW_TRY(upload(op, tw, &m.tw));
            EW_TRY(upload(op, tl, &m.tl));
            EW_TRY(upload(op, tu, &m.tu));
        }
        op->levels.push_back(L);
        op->mcoef.push_back(m);
        const double rho_j = stride == 1 ? fine.rho_j : stencil_rho_j(st);
        const bool can = (nl1 % 2 == 1) && (nl2 % 2 == 1) && nl1 >= 3 && nl2 >= 3;
        const bool enough = d.mg_max_levels == EW_MG_LEVELS_AUTO &&
                            std::pow(rho_j * rho_j, d.mg_coarse_sweeps) <= 0.1;
        if (!can || op->levels.size() >= max_levels || enough) break;
        Stencil9 next;
        galerkin(st, next);
        st = std::move(next);
        nl1 = (nl1 - 1) / 2;
        nl2 = (nl2 - 1) / 2;
        stride *= 2;
    }
    return EW_OK;
}

}  // namespace
}  // namespace ew

using namespace ew;

extern "C" ew_status ew_op_create_mapped(const ew_grid_desc* grid, const ew_op_desc* desc, const double* xy_host,
                                         void* hip_stream, ew_op* out) {
    if (!out) return fail(EW_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!xy_host) return fail(EW_ERR_INVALID_ARG, "mapped grid coordinates are null");
    EW_TRY(validate_descs(grid, desc));
    if (grid->dim != 2) return fail(EW_ERR_UNSUPPORTED, "mapped grids are two-dimensional");
    if (grid->order != 2) return fail(EW_ERR_UNSUPPORTED, "mapped grids use the order-2 operator");
    for (int e = 0; e < 2; ++e)
        if (grid->walls[0][e] != EW_WALL_DIRICHLET || grid->walls[1][e] != EW_WALL_DIRICHLET)
            return fail(EW_ERR_UNSUPPORTED, "mapped grids have Dirichlet walls");
    if (desc->precision != EW_PREC_FP64) return fail(EW_ERR_UNSUPPORTED, "mapped grids run in FP64");
    if (desc->ts == EW_TS_IMPLICIT && (desc->predictor == EW_PRED_PROJ || desc->predictor == EW_PRED_CNN))
        return fail(EW_ERR_UNSUPPORTED, "on mapped grids the implicit guesses are ZERO, SCALED or EXTRAP");
    const int n1 = (int)grid->n[0], n2 = (int)grid->n[1];
    Nodes nd;
    EW_TRY(node_metrics(xy_host, n1, n2, nd));
    HostCoef hc;
    level_coefficients(nd, 1, n1, n2, 0.0, hc);

    std::unique_ptr<ew_op_s> op(new ew_op_s());
    op->dim = 2;
    op->order = 2;
    op->n[0] = n1;
    op->n[1] = n2;
    op->n[2] = 1;
    op->h[0] = 1.0 / (n1 + 1);  // parameter-space spacings
    op->h[1] = 1.0 / (n2 + 1);
    op->desc = *desc;
    op->stream = (hipStream_t)hip_stream;
    op->implicit = desc->ts == EW_TS_IMPLICIT;
    op->g = make_geo(2, op->n, op->h, 0);
    op->N = op->g.size();
    EW_HIP_TRY(hipGetDevice(&op->device));
    op->mapped = true;
    op->map_rho = hc.rho;
    TimePlan tp;
    make_time_plan(2, 2, op->h, op->desc, tp, hc.rho);
    op->omega_used = tp.omega_used;
    op->t_final = tp.t_final;
    op->n_t = tp.n_t;
    op->dt = tp.dt;
    op->alpha_d = tp.alpha_d;
    op->c = tp.c;
    op->a = 0.5 * op->dt * op->dt;
    // line over-relaxation weights: 1 unless given (the best weight depends
    // on the map: on the skew map (1.3, 1.2) took fewer cycles, on an annulus
    // sector 1 did)
    op->relax = desc->mg_relax != 0.0 ? desc->mg_relax : 1.0;
    op->relax_coarse = desc->mg_relax_coarse != 0.0 ? desc->mg_relax_coarse : 1.0;
    EW_TRY(upload_level(op.get(), hc, op->mc));
    const int64_t N = op->N;
    EW_TRY(op->alloc((void**)&op->partial_dev, kRedBlocks * sizeof(double) * 4));
    EW_HIP_TRY(hipHostMalloc((void**)&op->partial_host, kRedBlocks * sizeof(double) * 4, hipHostMallocDefault));
    EW_TRY(op->alloc((void**)&op->wA, N * sizeof(double)));
    EW_TRY(op->alloc((void**)&op->wB, N * sizeof(double)));
    if (op->implicit) {
        EW_TRY(op->alloc((void**)&op->sbuf, N * sizeof(double)));
        level_coefficients(nd, 1, n1, n2, op->a, hc);  // the fine level's rho_j needs a, known only now
        EW_TRY(build_mapped_hierarchy(op.get(), nd, hc));
    } else {
        EW_TRY(op->alloc((void**)&op->c_dev, op->c.size() * sizeof(double)));
        EW_HIP_TRY(hipMemcpy(op->c_dev, op->c.data(), op->c.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    *out = op.release();
    return EW_OK;
}

extern "C" ew_status ew_op_mapped_rho(ew_op op, double* rho_host) {
    if (!op || !rho_host) return fail(EW_ERR_INVALID_ARG, "null argument");
    if (!op->mapped) return fail(EW_ERR_INVALID_ARG, "operator is not on a mapped grid");
    *rho_host = op->map_rho;
    return EW_OK;
}
