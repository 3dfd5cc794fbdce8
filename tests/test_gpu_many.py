"""Many eigenpairs at once (Sec. "Changing the number of requested
eigenpairs"; Krylov dimension 2k + 1): bases past 64 columns are
orthogonalised by block CGS2, bases past 320 columns are rotated with Q
streamed through LDS in slabs, and Stage 2 projects over hundreds of locked
vectors with the tridiagonal-QR routine.  Bar: every eigenvalue within 1e-10
relative of the closed-form spectrum and the whole wanted band present with
multiplicity (as for the other eigensolver tests), orthonormal eigenvectors,
and L_h residuals within a bound that follows from the implicit solves'
tolerance.  Each S v carries an error of about tau ||v|| (tau = multigrid
tolerance) spread over all modes; a Ritz vector of beta picks it up divided
by its distance |beta| from the damped high modes, and L_h multiplies it by
up to mu_max, so ||L z + mu z|| / (mu ||z||) <= C tau mu_max / (mu |beta|).
The wide bands here reach the lowest modes (beta(0) = -1/2), where that
exceeds 1e-8; the test takes C = 10 and never less than 1e-8."""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from tests.gpu_helpers import make_op, oracle_plan, say
from tests.test_gpu_eigs import check_result

pytestmark = pytest.mark.gpu


def check_many(P, r):
    check_result(P, r, res_tol=None)
    h, _ = oracle_plan(P)
    mu_max = float(D.mu_all(P.n, h, P.order).max())
    mu, beta, res = np.array(r.mu), np.abs(np.array(r.beta)), np.array(r.res)
    bound = np.maximum(1e-8, 10.0 * P.mg_tol * mu_max / (mu * beta))
    assert np.all(res <= bound), [(m, b, x) for m, b, x, y in zip(mu, beta, res, bound) if x > y]
    # the wanted count is met by pairs within that bound (the library's n_conv
    # counts the flat eig-res <= 1e-8, which the lowest modes need not reach)
    assert np.sum(res <= bound) >= P.k


@pytest.mark.parametrize("k", [48, 160])
def test_many_pairs_63(k):
    P = synthetic.config_many_pairs(k=k, n=63)
    op = make_op(P)
    say("many pairs 63^2 k", k, "m", P.m)
    r = op.eigs(P.k, P.m, seed=P.seed)
    check_many(P, r)
    Y = r.Y.cpu().numpy()
    assert np.max(np.abs(Y.T @ Y - np.eye(Y.shape[1]))) < 1e-9


def test_many_pairs_square128():
    P = synthetic.config_many_pairs(k=64)
    op = make_op(P)
    say("many pairs 127^2 k", P.k, "m", P.m)
    r = op.eigs(P.k, P.m, seed=P.seed, want_vectors=False)
    check_many(P, r)
    say("wave-solves", r.wave_solves, "converged", r.n_conv, "probes", r.probes)
