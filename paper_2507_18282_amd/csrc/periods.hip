// Choice of the number of filter periods N_p for a wanted number of
// eigenpairs (host only).  Longer integration narrows the main lobe of the
// filter function like 1/N_p, while the simultaneous-iteration rate estimate
// at the lobe's edge hardly depends on N_p; the most efficient runs keep about
// the wanted eigenvalues above beta ~ 0.8 (Sec. "Changing the number of filter
// periods"; Sec. "Estimating the EigenWave convergence rate").  The largest
// N_p whose lobe {beta >= beta_r} still holds k eigenvalues of the continuous
// box Laplacian is returned.
#include <cmath>
#include <vector>

#include "op.h"

namespace ew {
namespace {

double sinc(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }

// continuous filter function, three-sinc form (eq. filterThreeSincs)
double beta_cont(double lam, double omega, int n_p) {
    const double tf = n_p * 2.0 * M_PI / omega;
    return sinc((omega - lam) * tf) + sinc((omega + lam) * tf) - 0.5 * sinc(lam * tf);
}

// lambda = pi sqrt(sum_d (m_d / L_d)^2) <= lam_max, m_d >= 1, with multiplicity
void box_frequencies(int dim, const double* len, double lam_max, std::vector<double>& out) {
    int mmax[3] = {1, 1, 1};
    for (int d = 0; d < dim; ++d) mmax[d] = (int)std::floor(lam_max * len[d] / M_PI);
    out.clear();
    for (int d = 0; d < dim; ++d)
        if (mmax[d] < 1) return;
    const int mz = dim == 3 ? mmax[2] : 1;
    for (int k = 1; k <= mz; ++k)
        for (int j = 1; j <= mmax[1]; ++j)
            for (int i = 1; i <= mmax[0]; ++i) {
                double s = (i / len[0]) * (i / len[0]) + (j / len[1]) * (j / len[1]);
                if (dim == 3) s += (k / len[2]) * (k / len[2]);
                const double lam = M_PI * std::sqrt(s);
                if (lam <= lam_max) out.push_back(lam);
            }
}

int lobe(const std::vector<double>& lam, double omega, int n_p, double beta_r) {
    int c = 0;
    for (double l : lam)
        if (beta_cont(l, omega, n_p) >= beta_r) ++c;
    return c;
}

}  // namespace
}  // namespace ew

using namespace ew;

extern "C" ew_status ew_choose_periods(const ew_grid_desc* grid, const ew_op_desc* desc, int k, double beta_r,
                                       int np_max, int* n_p_out, int* n_lobe_out) {
    if (!grid || !desc) return fail(EW_ERR_INVALID_ARG, "null descriptor");
    if (grid->dim != 2 && grid->dim != 3) return fail(EW_ERR_INVALID_ARG, "dim must be 2 or 3");
    for (int d = 0; d < grid->dim; ++d) {
        if (!(grid->len[d] > 0.0)) return fail(EW_ERR_INVALID_ARG, "side lengths must be positive");
        if (grid->walls[d][0] != EW_WALL_DIRICHLET || grid->walls[d][1] != EW_WALL_DIRICHLET)
            return fail(EW_ERR_UNSUPPORTED, "the periods rule counts Dirichlet box modes");
    }
    if (!(desc->omega > 0.0)) return fail(EW_ERR_INVALID_ARG, "omega must be positive");
    if (desc->adjust_omega && desc->n_its < 5) return fail(EW_ERR_INVALID_ARG, "n_its must be >= 5");
    if (k < 1) return fail(EW_ERR_INVALID_ARG, "k must be positive");
    if (!(beta_r >= 0.5 && beta_r < 1.0)) return fail(EW_ERR_INVALID_ARG, "beta_r must be in [0.5, 1)");
    if (np_max < 1 || np_max > 4096) return fail(EW_ERR_INVALID_ARG, "np_max must be in [1, 4096]");
    double omega = desc->omega;
    if (desc->adjust_omega) {  // the frequency the operator's filter uses (eq. adjustedOmega)
        const double s = std::sin(M_PI / desc->n_its);
        omega = desc->omega * M_PI / desc->n_its * std::sqrt((1.0 - 2.0 * s * s) / (s * s));
    }
    const double lam_max = 1.5 * omega;
    double modes = 1.0;
    for (int d = 0; d < grid->dim; ++d) modes *= std::floor(lam_max * grid->len[d] / M_PI) + 1.0;
    if (modes > 5e7) return fail(EW_ERR_INVALID_ARG, "too many box modes below 1.5 omega to enumerate");
    std::vector<double> lam;
    box_frequencies(grid->dim, grid->len, lam_max, lam);
    int best = 1;
    for (int n_p = 1; n_p <= np_max; ++n_p) {
        if (lobe(lam, omega, n_p, beta_r) >= k) best = n_p;
        else break;
    }
    if (n_p_out) *n_p_out = best;
    if (n_lobe_out) *n_lobe_out = lobe(lam, omega, best, beta_r);
    return EW_OK;
}
