// Building blocks of the Arnoldi eigensolver shared by the single-problem
// (eigs.hip) and batched (batch.hip) drivers.
#pragma once

#include <vector>

#include "dense.h"
#include "ew_internal.h"

namespace ew {

struct Op;

constexpr int kGramBlocks = 256;

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
    double* h_dev = nullptr;   // Gram-Schmidt coefficients of one step
    double* q_dev = nullptr;   // small matrices for basis rotations
    double* gram_dev = nullptr;
    double* h_host = nullptr;
    std::vector<void*> owned;
    ~Workspace() {
        for (void* p : owned) hipFree(p);
        if (h_host) hipHostFree(h_host);
    }
    ew_status alloc(double** p, size_t count) {
        hipError_t e = hipMalloc((void**)p, count * sizeof(double) + 256);
        if (e != hipSuccess) return fail(EW_ERR_OOM, std::string("eigensolver workspace: ") + hipGetErrorString(e));
        owned.push_back(*p);
        return EW_OK;
    }
    // Allocate for Krylov dimension m and k wanted pairs.
    ew_status setup(int64_t n, int m_, int k) {
        N = n;
        m = m_;
        cap_lock = (int)std::min<int64_t>(std::min<int64_t>(N, 3 * m + k), 320);
        EW_TRY(alloc(&V, (size_t)N * (m + 1)));
        EW_TRY(alloc(&Vt, (size_t)N * (m + 1)));
        EW_TRY(alloc(&Y, (size_t)N * cap_lock));
        EW_TRY(alloc(&LY, (size_t)N * cap_lock));
        EW_TRY(alloc(&Z, (size_t)N * cap_lock));
        EW_TRY(alloc(&P, 2 * kRedBlocks));
        EW_TRY(alloc(&h_dev, 4 * 256 + 64));
        EW_TRY(alloc(&q_dev, (size_t)(4 * 256) * 256));
        EW_TRY(alloc(&gram_dev, (size_t)kGramBlocks * 32 * 32));
        EW_HIP_TRY(hipHostMalloc((void**)&h_host, (4 * 256 + 64) * sizeof(double), hipHostMallocDefault));
        return EW_OK;
    }
    double* col(double* base, int j) const { return base + (int64_t)j * N; }
};

// w <- w - sum_i (w, u_i) u_i by chained MGS links, then w <- w / ||w||;
// coeff receives the coefficients and the norm.  Host-blocking.
ew_status mgs_orthonormalize(Workspace& ws, double* w, const std::vector<const double*>& u, std::vector<double>& coeff);
// Y[:, 0:ncols] = X[:, 0:nx] Qm[0:nx, 0:ncols].  Host-blocking.
ew_status rotate(Workspace& ws, const double* X, int nx, const Mat& Qm, int ncols, double* Y);
int leading_converged(const std::vector<char>& conv);
ew_status stage2(Workspace& ws, int nl, const std::vector<double>& th_locked, double tol_res, int k_cap,
                 double* mu_host, double* beta_host, double* res_host, double* Y_dev, int* n_conv_out, int* n_ret_out,
                 double* max_res_out);

}  // namespace ew
