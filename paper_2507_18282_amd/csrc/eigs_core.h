// Building blocks of the Arnoldi eigensolver shared by the single-problem
// (eigs.hip) and batched (batch.hip) drivers.
#pragma once

#include <vector>

#include "dense.h"
#include "ew_internal.h"

namespace ew {

struct Op;

constexpr int kGramBlocks = 256;
constexpr size_t kHcolsMaxDoubles = (size_t)1 << 20;

// Device workspace of one eigenproblem.
struct Workspace {
    Op* op = nullptr;          // single-problem driver only
    hipStream_t stream = nullptr;
    Geo g{};
    int order = 2;
    int64_t N = 0;
    int m = 0, cap_lock = 0;
    double* V = nullptr;       // N x (m+1) Krylov basis
    double* Vt = nullptr;      // N x (m+1) rotation target
    double* Y = nullptr;       // N x cap_lock locked vectors
    double* LY = nullptr;      // N x cap_lock L_h applied to them / scratch
    double* Z = nullptr;       // N x cap_lock Rayleigh-Ritz vectors
    double* P = nullptr;       // 2 x kRedBlocks partial sums (ping-pong)
    double* h_dev = nullptr;   // Gram-Schmidt coefficients of one step (nu + 1)
    double* h_cur = nullptr;   // coefficients of one block Gram-Schmidt pass
    double* gs_partial = nullptr;  // block Gram-Schmidt dot partials
    double* gs_tmp = nullptr;      // block Gram-Schmidt column-chunk products
    double* q_dev = nullptr;   // small matrices for basis rotations
    double* gram_dev = nullptr;
    double* h_host = nullptr;
    double* hcols = nullptr;       // Gram-Schmidt coefficient columns of steps run without a round trip
    double* hcols_host = nullptr;  // (pinned) host copy of them
    int hcols_ld = 0;              // leading dimension (nu_max + 2)
    double* q_host = nullptr;      // pinned staging of rotation matrices (when small)
    hipEvent_t q_ev = nullptr;     // recorded after the last copy out of q_host
    size_t q_cap = 0;
    double* res_part = nullptr;    // Rayleigh-Ritz residual partials, 2 kRedBlocks per vector
    double* res_part_host = nullptr;
    int res_cap = 0;
    double* wtmp = nullptr;    // one vector for the weighted coordinates (Neumann walls, mapped grids)
    const double* wsq = nullptr;   // mapped grid: sqrt(J) and 1/sqrt(J) (the weights are J)
    const double* wisq = nullptr;
    int nu_max = 0;            // columns one orthogonalisation may involve
    std::vector<void*> owned;
    ~Workspace() {
        for (void* p : owned) dev_free(p);
        if (h_host) hipHostFree(h_host);
        if (hcols_host) hipHostFree(hcols_host);
        if (q_host) hipHostFree(q_host);
        if (q_ev) hipEventDestroy(q_ev);
        if (res_part_host) hipHostFree(res_part_host);
    }
    ew_status alloc(double** p, size_t count) {
        hipError_t e = dev_alloc((void**)p, count * sizeof(double) + 256, stream);
        if (e != hipSuccess) return fail(EW_ERR_OOM, std::string("eigensolver workspace: ") + hipGetErrorString(e));
        owned.push_back(*p);
        return EW_OK;
    }
    // Allocate for Krylov dimension m and k wanted pairs.  The locked set holds
    // up to 3m + k vectors, capped at max(320, m + k) (and at N).
    ew_status setup(int64_t n, int m_, int k) {
        N = n;
        m = m_;
        const int64_t cap = std::min<int64_t>(3 * (int64_t)m + k, std::max<int64_t>(320, (int64_t)m + k));
        cap_lock = (int)std::min<int64_t>(N, cap);
        nu_max = cap_lock + m + 2;
        const int64_t qdim = std::max<int64_t>(m + 1, cap_lock);
        EW_TRY(alloc(&V, (size_t)N * (m + 1)));
        EW_TRY(alloc(&Vt, (size_t)N * (m + 1)));
        EW_TRY(alloc(&Y, (size_t)N * cap_lock));
        EW_TRY(alloc(&LY, (size_t)N * cap_lock));
        EW_TRY(alloc(&Z, (size_t)N * cap_lock));
        EW_TRY(alloc(&P, 2 * kRedBlocks));
        const size_t hlen = std::max<size_t>((size_t)nu_max + 64, 2 * kRedBlocks + 64);  // also Stage-2 partials
        EW_TRY(alloc(&h_dev, hlen));
        EW_TRY(alloc(&q_dev, (size_t)qdim * qdim));
        EW_TRY(alloc(&gram_dev, (size_t)kGramBlocks * 32 * 32));
        if (g.wall || wsq) EW_TRY(alloc(&wtmp, (size_t)N));
        EW_HIP_TRY(hipHostMalloc((void**)&h_host, hlen * sizeof(double), hipHostMallocDefault));
        // Arnoldi steps queue their coefficients on the device and the host reads
        // a whole run of columns at once, when that buffer is small
        hcols_ld = nu_max + 2;
        const size_t hc = (size_t)m * hcols_ld;
        if (hc <= kHcolsMaxDoubles) {
            EW_TRY(alloc(&hcols, hc));
            EW_HIP_TRY(hipHostMalloc((void**)&hcols_host, hc * sizeof(double), hipHostMallocDefault));
        }
        // rotation matrices staged in pinned memory need no wait after their copy
        if ((size_t)qdim * qdim <= kHcolsMaxDoubles) {
            q_cap = (size_t)qdim * qdim;
            EW_HIP_TRY(hipHostMalloc((void**)&q_host, q_cap * sizeof(double), hipHostMallocDefault));
            EW_HIP_TRY(hipEventCreateWithFlags(&q_ev, hipEventDisableTiming));
        }
        return EW_OK;
    }
    // Buffers of the block Gram-Schmidt, allocated at its first use.
    ew_status setup_block_gs() {
        if (gs_tmp) return EW_OK;
        EW_TRY(alloc(&h_cur, (size_t)nu_max + 64));
        EW_TRY(alloc(&gs_partial, (size_t)kBlockGsMaxSlices * nu_max));
        EW_TRY(alloc(&gs_tmp, (size_t)kBlockGsTmpDoubles));
        return EW_OK;
    }
    double* col(double* base, int j) const { return base + (int64_t)j * N; }
};

// w <- w - sum_i (w, u_i) u_i by chained MGS links, then w <- w / ||w||;
// coeff receives the coefficients and the norm.  Host-blocking.
ew_status mgs_orthonormalize(Workspace& ws, double* w, const std::vector<const double*>& u, std::vector<double>& coeff);
// The same against the columns of [U1 (n1 columns) | U2 (n2 columns)]: up to
// kMgsMaxCols columns by MGS (in one workgroup for vectors of at most
// kMgsSmallMax points, else by chained links), block CGS2 beyond.
// Host-blocking; with coeff_dev != nullptr the n1 + n2 coefficients and the
// norm are left in coeff_dev on the device instead (nothing waits, coeff is
// untouched).
constexpr int kMgsMaxCols = 64;
ew_status orthonormalize(Workspace& ws, double* w, const double* u1, int n1, const double* u2, int n2,
                         std::vector<double>& coeff, double* coeff_dev = nullptr);
// out = W^{1/2} L_h W^{-1/2} in: the Laplacian in the eigensolver's
// coordinates, W the Neumann-wall weights or J on a mapped grid (plain L_h
// when there are none).  in and out may not alias.
ew_status apply_L_sym(Workspace& ws, const double* in, double* out);
// Y[:, 0:ncols] = X[:, 0:nx] Qm[0:nx, 0:ncols].  Host-blocking.
ew_status rotate(Workspace& ws, const double* X, int nx, const Mat& Qm, int ncols, double* Y);
int leading_converged(const std::vector<char>& conv);
ew_status stage2(Workspace& ws, int nl, const std::vector<double>& th_locked, double tol_res, int k_cap,
                 double* mu_host, double* beta_host, double* res_host, double* Y_dev, int* n_conv_out, int* n_ret_out,
                 double* max_res_out);

}  // namespace ew
