// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/eigenwave.h"

namespace ew {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error_cstr();
ew_status fail(ew_status code, const std::string& msg);

#define EW_HIP_TRY(expr)                                                        \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess)                                                   \
            return ::ew::fail(EW_ERR_HIP, std::string(#expr) + ": " +           \
                                              hipGetErrorString(e_));           \
    } while (0)

#define EW_TRY(expr)                         \
    do {                                     \
        ew_status s_ = (expr);               \
        if (s_ != EW_OK) return s_;          \
    } while (0)

// Device memory for the library's buffers: hipMalloc/hipFree, or the
// allocator installed with ew_set_allocator.  dev_free takes pointers from
// dev_alloc only.
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p);

// ---------------------------------------------------------------------------
// Grid geometry passed by value to kernels.  Interior points only, x fastest.
// ---------------------------------------------------------------------------
struct Geo {
    int dim;
    int nx, ny, nz;        // nz = 1 in 2D
    double ihx2, ihy2, ihz2;  // 1/h^2 per dimension (ihz2 = 0 in 2D)
    int wall;              // Neumann walls: bit 2d = low wall of dimension d, bit 2d+1 = high wall
    __host__ __device__ int64_t size() const { return (int64_t)nx * ny * nz; }
};

Geo make_geo(int dim, const int64_t* n, const double* h, int wall = 0);

// Number of partial sums written by the reduction kernels (one per block).
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// ---------------------------------------------------------------------------
// Kernel launchers (templated on the storage type T = double or float).
// All lengths are element counts; every launcher returns hipGetLastError().
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_laplacian(const T* u, T* out, const Geo& g, int order, hipStream_t s);

// out = W^{e/2} in, W = Neumann-wall weights (1/2 per Neumann wall of the
// point), e = +1 or -1; in and out may alias.
hipError_t launch_wall_scale(const double* in, double* out, const Geo& g, int e, hipStream_t s);

// Explicit leapfrog step fused with the filter accumulation.
//   first != 0: wnext = wcur + (dt2/2) L wcur;  acc = ccur*wcur + cnext*wnext
//   first == 0: wnext = 2 wcur - wprev + dt2 L wcur;  acc += cnext*wnext
// wnext may alias wprev.
template <typename T>
hipError_t launch_leapfrog(const T* wcur, const T* wprev, T* wnext, T* acc, const Geo& g, int order,
                           double dt2, double ccur, double cnext, int first, hipStream_t s);

// Implicit step update: wnext = sol - wprev; acc += cnext*wnext (wnext may alias wprev).
// With first != 0: wnext = sol; acc = ccur*wprev + cnext*wnext.
template <typename T, typename TA>
hipError_t launch_implicit_update(const T* sol, const T* wprev, T* wnext, TA* acc, int64_t n,
                                  double ccur, double cnext, int first, hipStream_t s);

// Multigrid pieces for M = I - a L.
// Out of place: xout = xin with the points of one colour relaxed,
// x + w (b - M x)_i / M_ii (w: relaxation weight).
template <typename T>
hipError_t launch_rb_half(const T* xin, T* xout, const T* b, double bscale, const Geo& g, int order, double a,
                          double w, int colour, hipStream_t s);
template <typename T>
hipError_t launch_prolong_correct(T* x, const T* xc, const Geo& gf, const Geo& gc, hipStream_t s);


// Elementwise helpers.
template <typename TD, typename TS>
hipError_t launch_convert(TD* dst, const TS* src, int64_t n, double scale, hipStream_t s);
template <typename T, typename TE>
hipError_t launch_add_inplace(T* x, const TE* e, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, int64_t n, T value, hipStream_t s);
template <typename T>
hipError_t launch_scale_copy(T* dst, const T* src, int64_t n, double scale, hipStream_t s);

// FP64 vector kernels for the Arnoldi process (deterministic block reductions).
hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* partial, hipStream_t s);
// MGS link: h = sum(partial_in); if (store_h) *h_out = h;
// w -= h * vprev; partial_out = partial dot(w, vnext) (vnext may be w itself).
hipError_t launch_mgs_link(double* w, const double* vprev, const double* vnext, int64_t n,
                           const double* partial_in, double* partial_out, double* h_out, hipStream_t s);
// v = w / sqrt(sum(partial_in)); *nrm_out = sqrt(sum(partial_in)).
hipError_t launch_normalize_from_partial(const double* w, double* v, int64_t n, const double* partial_in,
                                         double* nrm_out, hipStream_t s);
// Y[:, c] = sum_i V[:, i] * Q[i + c*ldq], c < ncols, i < nv (column-major, leading dim n).
hipError_t launch_tall_gemm(const double* V, int64_t n, int nv, const double* Q_dev, int ldq, int ncols, double* Y,
                            hipStream_t s);
// One classical Gram-Schmidt pass of w against the columns of [U1 | U2]
// (n1 + n2 columns of length n, column-major): h_cur = U^T w (h_tot = h_cur,
// or += with accumulate), then w -= U h_cur.  Buffers: partial holds
// nslices * (n1 + n2) doubles, tmp nchunks * n (<= kBlockGsTmpDoubles).
constexpr int kBlockGsMaxSlices = 256;
constexpr int kBlockGsMaxChunks = 128;
constexpr int64_t kBlockGsTmpDoubles = (int64_t)1 << 20;
struct BlockGsPlan {
    int64_t slice;
    int nslices;
    int chunk;
    int nchunks;
};
BlockGsPlan block_gs_plan(int64_t n, int nu);
hipError_t launch_block_gs_pass(const double* u1, int n1, const double* u2, int n2, double* w, int64_t n,
                                const BlockGsPlan& p, double* partial, double* h_cur, double* h_tot, int accumulate,
                                double* tmp, hipStream_t s);
// Modified Gram-Schmidt of w (n <= kMgsSmallMax points) against the columns of
// [U1 | U2] in one workgroup: h_out[0:n1+n2] = coefficients, h_out[n1+n2] =
// norm, w normalised.
constexpr int64_t kMgsSmallMax = 8192;  // 8 points per thread of 1024 (registers, no spills)
hipError_t launch_mgs_small(const double* u1, int n1, const double* u2, int n2, double* w, int64_t n, double* h_out,
                            hipStream_t s);
// Partial Gram blocks: block b writes P_b[i*nb + j] = sum over its rows of A[:,i]*B[:,j]
// (na, nb <= 32; partial holds nblocks*na*nb doubles).
hipError_t launch_gram_partial(const double* A, int na, const double* B, int nb, int64_t n, double* partial,
                               int nblocks, hipStream_t s);
// Partials of ||lz + mu z||^2 (partial[0:kRedBlocks]) and ||z||^2 (partial[kRedBlocks:2 kRedBlocks]).
hipError_t launch_eig_residual(const double* lz, const double* z, double mu, int64_t n, double* partial,
                               hipStream_t s);
// Per-block entry of largest magnitude (first index on ties): partial[0:kRedBlocks]
// values, partial[kRedBlocks:2 kRedBlocks] indices (as doubles, -1 for none).
hipError_t launch_absmax_partial(const double* y, int64_t n, double* partial, hipStream_t s);
hipError_t launch_splitmix_uniform(double* x, int64_t n, uint64_t seed, hipStream_t s);

// ---------------------------------------------------------------------------
// Single curvilinear grid (mapped.hip): device arrays of the order-2
// conservative operator, built once from the grid coordinates.  nx x ny
// active points, x fastest; half point i - 1/2 lies between nodes i - 1 and i.
// ---------------------------------------------------------------------------
struct MapCoef {
    const double* cw;   // (nx + 1) x ny: A11 / dr^2 at half point i - 1/2, index i + (nx + 1) j
    const double* cs;   // nx x (ny + 1): A22 / ds^2 at half point j - 1/2, index i + nx j
    const double* cb;   // nx x ny: J a^12 / (4 dr ds) at the node
    const double* ij;   // nx x ny: 1 / J
    const double* sq;   // nx x ny: sqrt(J)
    const double* isq;  // nx x ny: 1 / sqrt(J)
    // Thomas factors of M = I - a L_h restricted to each grid line of constant
    // j (multigrid levels only; null where lines are relaxed point-wise):
    // forward y_i = rhs_i tw_i - tl_i y_{i-1}, backward x_i = y_i - tu_i x_{i+1}
    const double* tw;   // nx x ny: 1 / pivot
    const double* tl;   // nx x ny: sub-diagonal entry / pivot (0 at i = 0)
    const double* tu;   // nx x ny: super-diagonal entry / pivot
    // Coarse multigrid levels: M itself as nine weights per point (Galerkin
    // product of the level above), gw[k nx ny + c] for the neighbour offsets
    // k = C, W, E, S, N, SW, SE, NW, NE; when set the kernels use these and
    // not the coefficient arrays above
    const double* gw;
};
hipError_t launch_laplacian_mapped(const double* u, double* out, const Geo& g, const MapCoef& m, hipStream_t s);
// Explicit leapfrog steps with the mapped operator fused with the filter
// accumulation, as launch_leapfrog: steps k0 .. k0 + ns - 1 of a wave-solve
// in one launch, 1 <= ns <= mapped_steps_per_launch(); reads
// W^{k0} (wcur) and W^{k0-1} (wprev, null for k0 = 0, when the first step's
// rule applies), writes W^{k0+ns} to dcur and W^{k0+ns-1} to dprev (neither
// may alias wcur or wprev) and accumulates cfil_dev[k + 1] W^{k+1} into acc
// (set to cfil_dev[0] W^0 + cfil_dev[1] W^1 when k0 = 0).
int mapped_steps_per_launch();
hipError_t launch_leapfrog_mapped_blocked(const double* wcur, const double* wprev, double* dcur, double* dprev,
                                          double* acc, const Geo& g, const MapCoef& m, double dt2,
                                          const double* cfil_dev, int k0, int ns, hipStream_t s);
// The same for a 2D box in FP64 (orders 2 and 4, any walls): steps k0 ..
// k0 + ns - 1 in one launch, 1 <= ns <= box_steps_per_launch(order).
int box_steps_per_launch(int order);
hipError_t launch_leapfrog_box_blocked(const double* wcur, const double* wprev, double* dcur, double* dprev,
                                       double* acc, const Geo& g, int order, double dt2, const double* cfil_dev,
                                       int k0, int ns, hipStream_t s);
// out = in * f elementwise (in and out may alias).
hipError_t launch_pointwise_mul(const double* in, const double* f, double* out, int64_t n, hipStream_t s);
// Multigrid for M = I - a L_h on a mapped level: out-of-place red-black
// half-sweep (the points of one colour relaxed from the input values, the
// others copied); residual r = bscale b - M x, stored when r_out != nullptr
// and with per-block partial sums of r^2 (kRedBlocks) when partial !=
// nullptr; full-weighting restriction of r to the level with n_c = (n - 1)/2.
// The half-sweep's correction is scaled by the weight w.
hipError_t launch_rb_half_mapped(const double* xin, double* xout, const double* b, double bscale, const Geo& g,
                                 const MapCoef& m, double a, double w, int colour, hipStream_t s);
// Zebra line relaxation, in place: every line j of parity `parity` solved
// exactly for its own points with the values on lines j +- 1 held, and the
// line set to x + w (solution - x) (needs m.tw and line_relax_fits(g.nx)).
bool line_relax_fits(int nx);
hipError_t launch_line_half_mapped(double* x, const double* b, double bscale, const Geo& g, const MapCoef& m,
                                   double a, double w, int parity, hipStream_t s);
hipError_t launch_residual_mapped(const double* x, const double* b, double bscale, const Geo& g, const MapCoef& m,
                                  double a, double* partial, double* r_out, hipStream_t s);
hipError_t launch_restrict_fw(const double* r, const Geo& gf, double* bc, const Geo& gc, hipStream_t s);

}  // namespace ew
