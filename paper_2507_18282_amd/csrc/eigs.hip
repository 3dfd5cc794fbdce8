// ew_eigs: restarted Arnoldi with modified Gram-Schmidt over the WaveHoltz
// operator S, Krylov-Schur restarting, deflation probes for repeated
// eigenvalues, and the Rayleigh-Ritz stage with L_h.
//
// Vectors live on the device; the host holds only the small projected
// matrices.  Arnoldi steps are queued back to back with their Gram-Schmidt
// coefficients left in device columns, which the host reads once per run of
// steps (at a restart or a probe's convergence test); when those columns would
// not fit a small buffer, each step crosses the host/device boundary once.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "eigs_core.h"
#include "op.h"

namespace ew {

constexpr int kMaxKrylov = 4096;

// w <- w - sum_i (w, u_i) u_i over the vector list by chained MGS links, then
// w <- w / ||w||.  hd (device) receives the n_u coefficients and the norm.
static ew_status mgs_chain(Workspace& ws, double* w, const std::vector<const double*>& u, double* hd) {
    hipStream_t s = ws.stream;
    const int nu = (int)u.size();
    double* P0 = ws.P;
    double* P1 = ws.P + kRedBlocks;
    if (nu == 0) {
        EW_HIP_TRY(launch_dot_partial(w, w, ws.N, P0, s));
        EW_HIP_TRY(launch_normalize_from_partial(w, w, ws.N, P0, hd, s));
    } else {
        EW_HIP_TRY(launch_dot_partial(w, u[0], ws.N, P0, s));
        for (int i = 1; i <= nu; ++i) {
            const double* pin = (i % 2 == 1) ? P0 : P1;
            double* pout = (i % 2 == 1) ? P1 : P0;
            const double* vnext = (i < nu) ? u[i] : w;
            EW_HIP_TRY(launch_mgs_link(w, u[i - 1], vnext, ws.N, pin, pout, hd + (i - 1), s));
        }
        const double* plast = (nu % 2 == 1) ? P1 : P0;
        EW_HIP_TRY(launch_normalize_from_partial(w, w, ws.N, plast, hd + nu, s));
    }
    return EW_OK;
}

static ew_status fetch_coeff(Workspace& ws, int nu, std::vector<double>& coeff) {
    EW_HIP_TRY(hipMemcpyAsync(ws.h_host, ws.h_dev, (nu + 1) * sizeof(double), hipMemcpyDeviceToHost, ws.stream));
    EW_HIP_TRY(hipStreamSynchronize(ws.stream));
    coeff.assign(ws.h_host, ws.h_host + nu + 1);
    for (double v : coeff)
        if (!std::isfinite(v)) return fail(EW_ERR_NONFINITE, "non-finite value in Gram-Schmidt");
    return EW_OK;
}

ew_status mgs_orthonormalize(Workspace& ws, double* w, const std::vector<const double*>& u, std::vector<double>& coeff) {
    EW_TRY(mgs_chain(ws, w, u, ws.h_dev));
    return fetch_coeff(ws, (int)u.size(), coeff);
}

ew_status orthonormalize(Workspace& ws, double* w, const double* u1, int n1, const double* u2, int n2,
                         std::vector<double>& coeff, double* coeff_dev) {
    const int nu = n1 + n2;
    double* hd = coeff_dev ? coeff_dev : ws.h_dev;
    if (ws.N <= kMgsSmallMax && nu <= kMgsMaxCols) {
        // short vectors, short basis: the whole modified Gram-Schmidt in one workgroup
        EW_HIP_TRY(launch_mgs_small(u1, n1, u2, n2, w, ws.N, hd, ws.stream));
    } else if (nu <= kMgsMaxCols) {
        std::vector<const double*> u;
        u.reserve(nu);
        for (int i = 0; i < n1; ++i) u.push_back(u1 + (int64_t)i * ws.N);
        for (int i = 0; i < n2; ++i) u.push_back(u2 + (int64_t)i * ws.N);
        EW_TRY(mgs_chain(ws, w, u, hd));
    } else {
        if (nu > ws.nu_max) return fail(EW_ERR_INVALID_ARG, "orthogonalisation basis exceeds the workspace");
        EW_TRY(ws.setup_block_gs());
        hipStream_t s = ws.stream;
        const BlockGsPlan plan = block_gs_plan(ws.N, nu);
        // CGS2: two passes, coefficients summed into hd[0:nu]
        for (int pass = 0; pass < 2; ++pass)
            EW_HIP_TRY(launch_block_gs_pass(u1, n1, u2, n2, w, ws.N, plan, ws.gs_partial, ws.h_cur, hd, pass,
                                            ws.gs_tmp, s));
        EW_HIP_TRY(launch_dot_partial(w, w, ws.N, ws.P, s));
        EW_HIP_TRY(launch_normalize_from_partial(w, w, ws.N, ws.P, hd + nu, s));
    }
    if (coeff_dev) return EW_OK;
    return fetch_coeff(ws, nu, coeff);
}

// Y[:, 0:ncols] = X[:, 0:nx] Qm[0:nx, 0:ncols] (Qm row-major nx x qcols).
// With the pinned staging buffer the call returns without waiting: the next
// call first waits for the event that marks this copy done.
ew_status rotate(Workspace& ws, const double* X, int nx, const Mat& Qm, int ncols, double* Y) {
    if (ws.q_host && (size_t)nx * ncols <= ws.q_cap) {
        EW_HIP_TRY(hipEventSynchronize(ws.q_ev));
        for (int c = 0; c < ncols; ++c)
            for (int i = 0; i < nx; ++i) ws.q_host[(size_t)c * nx + i] = Qm(i, c);
        EW_HIP_TRY(hipMemcpyAsync(ws.q_dev, ws.q_host, (size_t)nx * ncols * sizeof(double), hipMemcpyHostToDevice,
                                  ws.stream));
        EW_HIP_TRY(hipEventRecord(ws.q_ev, ws.stream));
        EW_HIP_TRY(launch_tall_gemm(X, ws.N, nx, ws.q_dev, nx, ncols, Y, ws.stream));
        return EW_OK;
    }
    std::vector<double> qc((size_t)nx * ncols);
    for (int c = 0; c < ncols; ++c)
        for (int i = 0; i < nx; ++i) qc[(size_t)c * nx + i] = Qm(i, c);
    EW_HIP_TRY(hipMemcpyAsync(ws.q_dev, qc.data(), qc.size() * sizeof(double), hipMemcpyHostToDevice, ws.stream));
    EW_HIP_TRY(launch_tall_gemm(X, ws.N, nx, ws.q_dev, nx, ncols, Y, ws.stream));
    // qc must outlive the copy: the stream is synchronised before it goes out of scope.
    EW_HIP_TRY(hipStreamSynchronize(ws.stream));
    return EW_OK;
}

int leading_converged(const std::vector<char>& conv) {
    int n = 0;
    while (n < (int)conv.size() && conv[n]) ++n;
    return n;
}

struct RunResult {
    std::vector<double> theta;
    Mat Q;                    // m x m, columns ordered by |theta| descending
    std::vector<char> conv;
};

// The eigensolver's coordinates: y = W^{1/2} u with W the Neumann-wall
// weights, or J on a mapped grid, in which S and L_h are symmetric (identity
// when there are neither).
static bool weighted(const Workspace& ws) { return ws.g.wall != 0 || ws.wsq != nullptr; }

// out = W^{e/2} in (in and out may alias)
static hipError_t weight_scale(const Workspace& ws, const double* in, double* out, int e) {
    if (ws.wsq) return launch_pointwise_mul(in, e > 0 ? ws.wsq : ws.wisq, out, ws.N, ws.stream);
    return launch_wall_scale(in, out, ws.g, e, ws.stream);
}

static hipError_t plain_laplacian(const Workspace& ws, const double* in, double* out) {
    if (ws.op && ws.op->mapped) return launch_laplacian_mapped(in, out, ws.g, ws.op->mc, ws.stream);
    return launch_laplacian<double>(in, out, ws.g, ws.order, ws.stream);
}

static ew_status apply_S_sym(Workspace& ws, const double* in, double* out) {
    Op* op = ws.op;
    if (!weighted(ws)) return op->apply_filter(in, out);
    EW_HIP_TRY(weight_scale(ws, in, ws.wtmp, -1));
    EW_TRY(op->apply_filter(ws.wtmp, out));
    EW_HIP_TRY(weight_scale(ws, out, out, 1));
    return EW_OK;
}

ew_status apply_L_sym(Workspace& ws, const double* in, double* out) {
    if (!weighted(ws)) {
        EW_HIP_TRY(plain_laplacian(ws, in, out));
        return EW_OK;
    }
    EW_HIP_TRY(weight_scale(ws, in, ws.wtmp, -1));
    EW_HIP_TRY(plain_laplacian(ws, ws.wtmp, out));
    EW_HIP_TRY(weight_scale(ws, out, out, 1));
    return EW_OK;
}

// With the environment variable EW_EIGS_PROGRESS set (to anything but "0"),
// every convergence test of a run prints one line to stderr, so that a long
// solve on a large grid shows how far it has come.
static bool progress_enabled() {
    const char* e = std::getenv("EW_EIGS_PROGRESS");
    return e != nullptr && e[0] != '\0' && std::strcmp(e, "0") != 0;
}

// Probe runs test for convergence before the basis is full, at basis sizes
// from kProbeFirstCheck on that are a power of two or three times one (16,
// 24, 32, 48, 64, ...; the last test is always at the full basis).
constexpr int kProbeFirstCheck = 16;
static bool probe_check_size(int s) {
    if (s < kProbeFirstCheck) return false;
    while ((s & 1) == 0) s >>= 1;
    return s == 1 || s == 3;
}

// One Krylov-Schur run on S deflated by the nl locked vectors, started from
// column 0 of ws.V (already filled, not yet orthonormalised).
//
// Stopping rules: the first run stops when its k leading Ritz pairs (by
// |theta|) have converged.  A probe run (probe > 0, deflation probes for
// repeated eigenvalues) stops when every Ritz value with |theta| >= floor_abs
// has converged, or when no eigenvalue of the deflated operator is left at or
// above the floor: the leading Ritz value has converged below it, or both
// extreme Ritz values, widened by their residual bounds, lie below it
// (tested from min(kProbeFirstCheck, m) basis vectors on; a Krylov space's
// extreme Ritz values approach the extreme eigenvalues first).
ew_status ks_run(Workspace& ws, int nl, int n_keep, double tol_ritz, int probe, int k, double floor_abs,
                 int64_t ws_budget, uint64_t seed_base, int64_t& wave_solves, int64_t& restarts, RunResult& out) {
    Op* op = ws.op;
    const int m = ws.m;
    Mat T(m + 1, m);
    std::vector<double> coeff, res;
    // Ritz pairs of the leading s x s projected matrix (symmetric up to
    // rounding): out.theta, out.Q (s x s, columns by |theta| descending),
    // residual bounds res and out.conv.
    auto ritz = [&](int s) {
        Mat A(s, s);
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) A(i, j) = 0.5 * (T(i, j) + T(j, i));
        std::vector<double> w0;
        Mat Q0;
        sym_eigh(A, w0, Q0);
        std::vector<int> idx = order_by_abs_desc(w0);
        out.theta.assign(s, 0.0);
        out.Q = Mat(s, s);
        for (int c = 0; c < s; ++c) {
            out.theta[c] = w0[idx[c]];
            for (int i = 0; i < s; ++i) out.Q(i, c) = Q0(i, idx[c]);
        }
        const double beta_s = T(s, s - 1);
        res.assign(s, 0.0);
        out.conv.assign(s, 0);
        for (int c = 0; c < s; ++c) {
            res[c] = std::fabs(beta_s * out.Q(s - 1, c));
            out.conv[c] = res[c] <= tol_ritz * std::fabs(out.theta[c]);
        }
    };
    auto stop_rule = [&](int s) -> bool {
        const int nlead = leading_converged(out.conv);
        if (probe == 0) return nlead >= k;
        if (s >= std::min(kProbeFirstCheck, m)) {
            int cmax = 0, cmin = 0;
            for (int c = 1; c < s; ++c) {
                if (out.theta[c] > out.theta[cmax]) cmax = c;
                if (out.theta[c] < out.theta[cmin]) cmin = c;
            }
            const double top = std::max(std::fabs(out.theta[cmax]) + res[cmax], std::fabs(out.theta[cmin]) + res[cmin]);
            if (top < floor_abs) return true;
        }
        if (!out.conv[0]) return false;
        if (std::fabs(out.theta[0]) < floor_abs) return true;
        int n_band = 0;
        for (int c = 0; c < s; ++c) n_band += std::fabs(out.theta[c]) >= floor_abs;
        return nlead >= n_band;
    };
    // normalise the start vector against the locked set
    EW_TRY(orthonormalize(ws, ws.col(ws.V, 0), ws.Y, nl, nullptr, 0, coeff));
    if (!std::isfinite(coeff.back())) return fail(EW_ERR_NONFINITE, "non-finite start vector");
    if (!(coeff.back() > 0.0)) return fail(EW_ERR_NONFINITE, "start vector lies in the locked space");
    // probe runs test for convergence after the steps that reach these basis sizes
    auto probe_check_at = [&](int s) {
        return probe > 0 && s < m && probe_check_size(s);
    };
    auto budget_hit = [&]() {
        // Budget reached inside a cycle: report no converged pairs.
        out.theta.clear();
        out.conv.clear();
        out.Q = Mat(m, m);
    };
    // One Arnoldi step j with the coefficients read back at once; a breakdown
    // (the Krylov space is invariant) continues from a fresh random direction
    // orthogonal to everything so far.
    auto sync_step = [&](int j) -> ew_status {
        double* w = ws.col(ws.V, j + 1);
        EW_TRY(apply_S_sym(ws, ws.col(ws.V, j), w));
        ++wave_solves;
        EW_TRY(orthonormalize(ws, w, ws.Y, nl, ws.V, j + 1, coeff));
        double hsq = 0.0;
        for (int i = 0; i <= j; ++i) {
            T(i, j) = coeff[nl + i];
            hsq += coeff[nl + i] * coeff[nl + i];
        }
        double nrm = coeff.back();
        if (!(nrm > 1e-12 * std::sqrt(hsq + nrm * nrm))) {
            EW_HIP_TRY(launch_splitmix_uniform(w, ws.N, seed_base + 0x100000ULL + (uint64_t)wave_solves, op->stream));
            EW_TRY(orthonormalize(ws, w, ws.Y, nl, ws.V, j + 1, coeff));
            nrm = 0.0;
        }
        T(j + 1, j) = nrm;
        return EW_OK;
    };
    const bool progress = progress_enabled();
    auto report = [&](int s) {
        if (!progress) return;
        std::fprintf(stderr,
                     "ew_eigs: run %d, basis %d, %lld wave-solves, %lld restarts, %d leading Ritz pairs converged\n",
                     probe, s, (long long)wave_solves, (long long)restarts, leading_converged(out.conv));
        std::fflush(stderr);
    };
    int p = 0;
    for (;;) {
        int j = p;
        while (j < m) {
            if (wave_solves >= ws_budget) {
                budget_hit();
                return EW_OK;
            }
            int jend = j + 1;  // steps j .. jend-1 run before the host looks at their coefficients
            if (ws.hcols) {
                jend = m;
                for (int s = j + 1; s < m; ++s)
                    if (probe_check_at(s)) {
                        jend = s;
                        break;
                    }
                jend = (int)std::min<int64_t>(jend, j + (ws_budget - wave_solves));
            }
            if (!ws.hcols || jend == j + 1) {
                EW_TRY(sync_step(j));
                ++j;
            } else {
                // Steps queued back to back: each leaves its coefficients in its
                // own column of ws.hcols, read once at the end of the run.
                for (int jj = j; jj < jend; ++jj) {
                    EW_TRY(apply_S_sym(ws, ws.col(ws.V, jj), ws.col(ws.V, jj + 1)));
                    ++wave_solves;
                    EW_TRY(orthonormalize(ws, ws.col(ws.V, jj + 1), ws.Y, nl, ws.V, jj + 1, coeff,
                                          ws.hcols + (size_t)(jj - j) * ws.hcols_ld));
                }
                EW_HIP_TRY(hipMemcpyAsync(ws.hcols_host, ws.hcols, (size_t)(jend - j) * ws.hcols_ld * sizeof(double),
                                          hipMemcpyDeviceToHost, op->stream));
                EW_HIP_TRY(hipStreamSynchronize(op->stream));
                // the first step with a non-finite coefficient or a breakdown (later
                // columns may carry what it spread) is redone on the host path
                int broke = -1;
                for (int jj = j; jj < jend && broke < 0; ++jj) {
                    const double* c = ws.hcols_host + (size_t)(jj - j) * ws.hcols_ld;
                    const int nu = nl + jj + 1;
                    for (int i = 0; i <= nu && broke < 0; ++i)
                        if (!std::isfinite(c[i])) broke = jj;
                    if (broke >= 0) break;
                    double hsq = 0.0;
                    for (int i = 0; i <= jj; ++i) {
                        T(i, jj) = c[nl + i];
                        hsq += c[nl + i] * c[nl + i];
                    }
                    const double nrm = c[nu];
                    if (!(nrm > 1e-12 * std::sqrt(hsq + nrm * nrm))) broke = jj;
                    else T(jj + 1, jj) = nrm;
                }
                if (broke < 0) {
                    j = jend;
                } else {
                    // same inputs as before (the basis up to column broke is
                    // unchanged); a non-finite value there is reported as such.
                    // The queued steps from broke on are discarded: they leave
                    // the count of kept Arnoldi steps and are run again.
                    wave_solves -= jend - broke;
                    EW_TRY(sync_step(broke));
                    j = broke + 1;
                    continue;
                }
            }
            const int s = j;
            if (probe_check_at(s)) {
                ritz(s);
                const bool stop = stop_rule(s);
                report(s);
                if (stop) return EW_OK;
            }
        }
        ritz(m);
        const double beta_m = T(m, m - 1);
        const bool stop = stop_rule(m);
        report(m);
        if (stop || wave_solves >= ws_budget) return EW_OK;
        // Thick restart: keep the leading n_keep Ritz vectors and the residual vector.
        EW_TRY(rotate(ws, ws.V, m, out.Q, n_keep, ws.Vt));
        EW_HIP_TRY(hipMemcpyAsync(ws.col(ws.Vt, n_keep), ws.col(ws.V, m), ws.N * sizeof(double),
                                  hipMemcpyDeviceToDevice, op->stream));
        std::swap(ws.V, ws.Vt);
        T = Mat(m + 1, m);
        for (int c = 0; c < n_keep; ++c) {
            T(c, c) = out.theta[c];
            T(n_keep, c) = beta_m * out.Q(m - 1, c);
        }
        p = n_keep;
        ++restarts;
    }
}

// Sum nblocks partial Gram blocks on the host, in block order.
ew_status gram(Workspace& ws, const double* A, int na, const double* B, int nb, Mat& G, int r0, int c0) {
    EW_HIP_TRY(launch_gram_partial(A, na, B, nb, ws.N, ws.gram_dev, kGramBlocks, ws.stream));
    std::vector<double> hbuf((size_t)kGramBlocks * na * nb);
    EW_HIP_TRY(hipMemcpyAsync(hbuf.data(), ws.gram_dev, hbuf.size() * sizeof(double), hipMemcpyDeviceToHost,
                              ws.stream));
    EW_HIP_TRY(hipStreamSynchronize(ws.stream));
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            double s = 0.0;
            for (int b = 0; b < kGramBlocks; ++b) s += hbuf[(size_t)b * na * nb + i * nb + j];
            G(r0 + i, c0 + j) = s;
        }
    return EW_OK;
}

ew_status full_gram(Workspace& ws, const double* A, const double* B, int n, Mat& G) {
    G = Mat(n, n);
    for (int i0 = 0; i0 < n; i0 += 32)
        for (int j0 = 0; j0 < n; j0 += 32)
            EW_TRY(gram(ws, ws.col(const_cast<double*>(A), i0), std::min(32, n - i0),
                        ws.col(const_cast<double*>(B), j0), std::min(32, n - j0), G, i0, j0));
    return EW_OK;
}

}  // namespace ew

namespace ew {

// Stage 2: Rayleigh-Ritz of L_h on the nl locked vectors Y (eq.
// discreteRayleighQuotient applied blockwise): G q = mu B q with G = -Y^T L Y
// and B = Y^T Y; residuals ||L z + mu z|| / (mu ||z||); pairs written ordered by
// |beta| descending, beta of each Rayleigh-Ritz vector being the locked Ritz
// values averaged with weights q_i^2.
ew_status stage2(Workspace& ws, int nl, const std::vector<double>& th_locked, double tol_res, int k_cap,
                 double* mu_host, double* beta_host, double* res_host, double* Y_dev, int* n_conv_out, int* n_ret_out,
                 double* max_res_out) {
    const int64_t N = ws.N;
    for (int i = 0; i < nl; ++i)
        EW_TRY(apply_L_sym(ws, ws.col(ws.Y, i), ws.col(ws.LY, i)));
    Mat G, B;
    EW_TRY(full_gram(ws, ws.Y, ws.LY, nl, G));
    EW_TRY(full_gram(ws, ws.Y, ws.Y, nl, B));
    Mat Gs(nl, nl), Bs(nl, nl);
    for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j) {
            Gs(i, j) = -0.5 * (G(i, j) + G(j, i));
            Bs(i, j) = 0.5 * (B(i, j) + B(j, i));
        }
    Mat Lc;
    if (!cholesky(Bs, Lc)) return fail(EW_ERR_NONFINITE, "locked vectors are not linearly independent");
    Mat Li = lower_inverse(Lc);
    // C = Li Gs Li^T as two products, then Q = Li^T Zc
    Mat T1(nl, nl), C(nl, nl);
    for (int i = 0; i < nl; ++i) {
        double* t = &T1.a[(size_t)i * nl];
        for (int a = 0; a <= i; ++a) {
            const double l = Li(i, a);
            const double* g = &Gs.a[(size_t)a * nl];
            for (int b = 0; b < nl; ++b) t[b] += l * g[b];
        }
    }
    for (int i = 0; i < nl; ++i)
        for (int j = 0; j <= i; ++j) {
            const double* t = &T1.a[(size_t)i * nl];
            const double* l = &Li.a[(size_t)j * nl];
            double s = 0.0;
            for (int b = 0; b <= j; ++b) s += t[b] * l[b];
            C(i, j) = C(j, i) = s;
        }
    std::vector<double> mu;
    Mat Zc;
    sym_eigh(C, mu, Zc);
    Mat Qr(nl, nl);  // Q = Li^T Zc
    for (int a = 0; a < nl; ++a) {
        const double* z = &Zc.a[(size_t)a * nl];
        for (int i = 0; i <= a; ++i) {
            const double l = Li(a, i);
            double* q = &Qr.a[(size_t)i * nl];
            for (int j = 0; j < nl; ++j) q[j] += l * z[j];
        }
    }
    // beta of each Rayleigh-Ritz vector: theta averaged with weights Q^2
    std::vector<double> beta(nl);
    for (int j = 0; j < nl; ++j) {
        double num = 0.0, den = 0.0;
        for (int i = 0; i < nl; ++i) {
            num += th_locked[i] * Qr(i, j) * Qr(i, j);
            den += Qr(i, j) * Qr(i, j);
        }
        beta[j] = num / den;
    }
    EW_TRY(rotate(ws, ws.Y, nl, Qr, nl, ws.Z));
    std::vector<double> res(nl), znorm(nl);
    // L z_j into the (no longer needed) L Y buffer and the partials of
    // ||L z + mu z|| and ||z|| for every j, read back once
    if (ws.res_cap < nl) {
        EW_TRY(ws.alloc(&ws.res_part, (size_t)nl * 2 * kRedBlocks));
        if (ws.res_part_host) hipHostFree(ws.res_part_host);
        ws.res_part_host = nullptr;
        EW_HIP_TRY(hipHostMalloc((void**)&ws.res_part_host, (size_t)nl * 2 * kRedBlocks * sizeof(double),
                                 hipHostMallocDefault));
        ws.res_cap = nl;
    }
    for (int j = 0; j < nl; ++j) {
        EW_TRY(apply_L_sym(ws, ws.col(ws.Z, j), ws.col(ws.LY, j)));
        EW_HIP_TRY(launch_eig_residual(ws.col(ws.LY, j), ws.col(ws.Z, j), mu[j], N,
                                       ws.res_part + (size_t)j * 2 * kRedBlocks, ws.stream));
    }
    EW_HIP_TRY(hipMemcpyAsync(ws.res_part_host, ws.res_part, (size_t)nl * 2 * kRedBlocks * sizeof(double),
                              hipMemcpyDeviceToHost, ws.stream));
    EW_HIP_TRY(hipStreamSynchronize(ws.stream));
    for (int j = 0; j < nl; ++j) {
        const double* hp = ws.res_part_host + (size_t)j * 2 * kRedBlocks;
        double r2 = 0.0, z2 = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) r2 += hp[b];
        for (int b = 0; b < kRedBlocks; ++b) z2 += hp[kRedBlocks + b];
        znorm[j] = std::sqrt(z2);
        // relative to mu; absolute for |mu| < 1 (the constant mode of a box
        // with Neumann walls only has mu = 0)
        res[j] = std::sqrt(r2) / (std::max(std::fabs(mu[j]), 1.0) * znorm[j]);
    }
    std::vector<int> order = order_by_abs_desc(beta);
    int n_conv = 0;
    for (int j = 0; j < nl; ++j) n_conv += res[j] <= tol_res;
    const int n_ret = std::min(nl, k_cap);
    double max_res = 0.0;
    for (int r = 0; r < n_ret; ++r) {
        const int j = order[r];
        mu_host[r] = mu[j];
        beta_host[r] = beta[j];
        res_host[r] = res[j];
        max_res = std::max(max_res, res[j]);
        if (Y_dev && !weighted(ws)) {
            EW_HIP_TRY(launch_scale_copy<double>(Y_dev + (int64_t)r * N, ws.col(ws.Z, j), N, 1.0 / znorm[j], ws.stream));
        } else if (Y_dev) {
            // back to the grid function u = W^{-1/2} z, unit 2-norm
            double* y = Y_dev + (int64_t)r * N;
            EW_HIP_TRY(weight_scale(ws, ws.col(ws.Z, j), y, -1));
            EW_HIP_TRY(launch_dot_partial(y, y, N, ws.P, ws.stream));
            EW_HIP_TRY(launch_normalize_from_partial(y, y, N, ws.P, nullptr, ws.stream));
        }
    }
    if (Y_dev && n_ret > 0) {
        // sign: the entry of largest magnitude (the first such) is positive
        for (int r = 0; r < n_ret; ++r)
            EW_HIP_TRY(launch_absmax_partial(Y_dev + (int64_t)r * N, N, ws.res_part + (size_t)r * 2 * kRedBlocks,
                                             ws.stream));
        EW_HIP_TRY(hipMemcpyAsync(ws.res_part_host, ws.res_part, (size_t)n_ret * 2 * kRedBlocks * sizeof(double),
                                  hipMemcpyDeviceToHost, ws.stream));
        EW_HIP_TRY(hipStreamSynchronize(ws.stream));
        for (int r = 0; r < n_ret; ++r) {
            const double* hp = ws.res_part_host + (size_t)r * 2 * kRedBlocks;
            double bv = 0.0, bi = -1.0;
            for (int b = 0; b < kRedBlocks; ++b) {
                const double v = hp[b], i = hp[kRedBlocks + b];
                if (i < 0.0) continue;
                if (bi < 0.0 || std::fabs(v) > std::fabs(bv) || (std::fabs(v) == std::fabs(bv) && i < bi)) {
                    bv = v;
                    bi = i;
                }
            }
            if (bv < 0.0)
                EW_HIP_TRY(launch_scale_copy<double>(Y_dev + (int64_t)r * N, Y_dev + (int64_t)r * N, N, -1.0,
                                                     ws.stream));
        }
    }
    EW_HIP_TRY(hipStreamSynchronize(ws.stream));
    *n_conv_out = n_conv;
    *n_ret_out = n_ret;
    *max_res_out = max_res;
    return EW_OK;
}

}  // namespace ew

using namespace ew;

extern "C" ew_status ew_eigs(ew_op op, const ew_eigs_desc* desc, int k_cap, double* mu_host, double* beta_host,
                             double* res_host, double* Y_dev, ew_eigs_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!op || !desc) return fail(EW_ERR_INVALID_ARG, "null argument");
    const int k = desc->k, m = desc->m;
    const int64_t N = op->N;
    if (k < 1 || m <= k || m > kMaxKrylov || (int64_t)m > N)
        return fail(EW_ERR_INVALID_ARG, "need 1 <= k < m <= min(" + std::to_string(kMaxKrylov) + ", n_active)");
    if (!(desc->tol_ritz > 0.0) || !(desc->tol_res > 0.0)) return fail(EW_ERR_INVALID_ARG, "tolerances must be > 0");
    if (desc->max_wave_solves < 1) return fail(EW_ERR_INVALID_ARG, "max_wave_solves must be >= 1");
    if (k_cap < 0 || (k_cap > 0 && (!mu_host || !beta_host || !res_host)))
        return fail(EW_ERR_INVALID_ARG, "k_cap > 0 needs mu_host, beta_host and res_host");
    int n_keep = desc->n_keep > 0 ? desc->n_keep : std::max(k, (m + k) / 2);
    n_keep = std::min(n_keep, m - 1);
    if (n_keep < k) return fail(EW_ERR_INVALID_ARG, "n_keep must be >= k");
    const int max_probes = desc->max_probes > 0 ? desc->max_probes : 16;

    Workspace ws;
    ws.op = op;
    ws.stream = op->stream;
    ws.g = op->g;
    ws.order = op->order;
    if (op->mapped) {
        ws.wsq = op->mc.sq;
        ws.wisq = op->mc.isq;
    }
    EW_TRY(ws.setup(N, m, k));

    const ew_op_stats s0 = op->stats;
    int64_t wave_solves = 0, restarts = 0;
    int nl = 0;
    std::vector<double> th_locked;
    int probe = 0, runs = 0;
    bool budget_hit = false;
    for (; probe < max_probes; ++probe) {
        // start vector
        if (probe == 0 && desc->v0_dev) {
            EW_HIP_TRY(hipMemcpyAsync(ws.V, desc->v0_dev, N * sizeof(double), hipMemcpyDeviceToDevice, op->stream));
        } else {
            EW_HIP_TRY(launch_splitmix_uniform(ws.V, N, desc->seed + (uint64_t)probe, op->stream));
        }
        double floor_abs = 0.0;
        if (probe > 0) {
            std::vector<double> a(th_locked.size());
            for (size_t i = 0; i < a.size(); ++i) a[i] = std::fabs(th_locked[i]);
            std::sort(a.begin(), a.end(), std::greater<double>());
            floor_abs = (1.0 - 1e-10) * a[k - 1];
        }
        RunResult rr;
        EW_TRY(ks_run(ws, nl, n_keep, desc->tol_ritz, probe, k, floor_abs, desc->max_wave_solves, desc->seed,
                      wave_solves, restarts, rr));
        ++runs;
        if (wave_solves >= desc->max_wave_solves) budget_hit = true;
        if (rr.theta.empty()) break;  // stopped by the budget inside a cycle
        int nlead = leading_converged(rr.conv);
        if (probe == 0 && nlead < k) break;  // budget exhausted before the first k converged
        if (probe > 0) {
            if (!rr.conv[0] || std::fabs(rr.theta[0]) < floor_abs) {
                if (rr.conv[0]) budget_hit = false;  // search complete
                break;
            }
            int n_band = 0;
            for (int c = 0; c < m; ++c) n_band += std::fabs(rr.theta[c]) >= floor_abs;
            nlead = std::min(nlead, n_band);
        }
        nlead = std::min(nlead, ws.cap_lock - nl);
        if (nlead <= 0) break;
        EW_TRY(rotate(ws, ws.V, rr.Q.n, rr.Q, nlead, ws.col(ws.Y, nl)));
        for (int c = 0; c < nlead; ++c) th_locked.push_back(rr.theta[c]);
        nl += nlead;
        if (budget_hit || nl >= ws.cap_lock) break;
    }

    if (nl < k) {
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->wave_solves = wave_solves;
            stats->restarts = restarts;
            stats->probes = runs;
            stats->time_steps = op->stats.time_steps - s0.time_steps;
            stats->pt_updates = op->stats.pt_updates - s0.pt_updates;
            stats->mg_cycles = op->stats.mg_cycles - s0.mg_cycles;
            EW_HIP_TRY(hipStreamSynchronize(op->stream));
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return fail(EW_ERR_NOT_CONVERGED, "eigensolver reached max_wave_solves with " + std::to_string(nl) +
                                              " converged pairs");
    }

    int n_conv = 0, n_ret = 0;
    double max_res = 0.0;
    EW_TRY(stage2(ws, nl, th_locked, desc->tol_res, k_cap, mu_host, beta_host, res_host, Y_dev, &n_conv, &n_ret,
                  &max_res));
    if (stats) {
        stats->n_conv = n_conv;
        stats->n_returned = n_ret;
        stats->wave_solves = wave_solves;
        stats->restarts = restarts;
        stats->probes = runs;
        stats->time_steps = op->stats.time_steps - s0.time_steps;
        stats->pt_updates = op->stats.pt_updates - s0.pt_updates;
        stats->mg_cycles = op->stats.mg_cycles - s0.mg_cycles;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->max_res = max_res;
    }
    if (budget_hit) return fail(EW_ERR_NOT_CONVERGED, "eigensolver reached max_wave_solves");
    return EW_OK;
}

extern "C" ew_status ew_sym_eig(int n, const double* a_host, double* w_host, double* q_host) {
    if (n < 1 || n > 8192 || !a_host || !w_host) return fail(EW_ERR_INVALID_ARG, "need 1 <= n <= 8192 and a, w");
    Mat A(n, n);
    std::memcpy(A.a.data(), a_host, (size_t)n * n * sizeof(double));
    std::vector<double> w;
    Mat Q;
    sym_eigh(A, w, Q);
    std::memcpy(w_host, w.data(), (size_t)n * sizeof(double));
    if (q_host) std::memcpy(q_host, Q.a.data(), (size_t)n * n * sizeof(double));
    return EW_OK;
}

extern "C" ew_status ew_fill_uniform(double* x_dev, int64_t n, uint64_t seed, void* hip_stream) {
    if (!x_dev || n < 0) return fail(EW_ERR_INVALID_ARG, "bad argument");
    if (n == 0) return EW_OK;
    EW_HIP_TRY(launch_splitmix_uniform(x_dev, n, seed, (hipStream_t)hip_stream));
    return EW_OK;
}

extern "C" const char* ew_last_error(void) { return ew::last_error_cstr(); }

extern "C" const char* ew_version(void) { return "eigenwave-mi355x 0.1 (gfx950)"; }
