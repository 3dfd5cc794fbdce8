"""Eigen drivers over the WaveHoltz operator S, and the Rayleigh quotient stage.

Test infrastructure only (see ``oracle/__init__``).

* :func:`power_iteration` -- Alg. 1 (EigenWave power iteration).
* :func:`arnoldi` -- Alg. 3 (Arnoldi with modified Gram-Schmidt).
* :func:`krylov_schur` -- Arnoldi with Krylov-Schur restarting (the restarted
  form of Alg. 3 the paper runs through SLEPc; wanted set = largest |theta|,
  the paper's "largestAbs") followed by Stage 2: a Rayleigh-Ritz projection of
  L_h onto the converged Ritz vectors (eq. discreteRayleighQuotient applied
  blockwise).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

Op = Callable[[np.ndarray], np.ndarray]


def power_iteration(apply_S: Op, apply_L: Op, v0: np.ndarray, tol: float, max_its: int = 10000):
    """Alg. 1: v <- S v, beta = (S v, v), normalise, stop when
    ||v_new - sign(beta) v|| < tol; lambda^2 from the Rayleigh quotient with L.
    Returns (mu, beta, v, iterations) with mu = lambda^2."""
    v = v0 / np.linalg.norm(v0)
    beta = 0.0
    its = 0
    for its in range(1, max_its + 1):
        w = apply_S(v)
        beta = float(np.dot(w, v))
        w = w / np.linalg.norm(w)
        done = np.linalg.norm(w - np.sign(beta) * v) < tol
        v = w
        if done:
            break
    mu = -float(np.dot(v, apply_L(v))) / float(np.dot(v, v))
    return mu, beta, v, its


def arnoldi(apply_A: Op, v: np.ndarray, m: int):
    """Alg. 3: m Arnoldi steps with modified Gram-Schmidt.

    Returns V (N x (m+1)) with orthonormal columns and H ((m+1) x m) upper
    Hessenberg with A V[:, :m] = V H.  (The paper's listing writes ``A v`` and
    ``h_{j+1,i}``; they are read as A v_j and h_{j+1,j}.)"""
    N = v.size
    V = np.zeros((N, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        w = apply_A(V[:, j])
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[:, i])
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    return V, H


def rayleigh_ritz_L(apply_L: Op, Y: np.ndarray):
    """Stage 2 over the columns of Y: project L_h onto span(Y) and diagonalise.

    Returns (mu, Z, res) with mu = lambda^2 ascending-by-index of input order
    unchanged semantics: Z = Y Q are the rotated vectors, mu_i = -(z_i, L z_i),
    res_i = ||L z_i + mu_i z_i||_2 / (mu_i ||z_i||_2).  For one vector this is
    the Rayleigh quotient of eq. discreteRayleighQuotient with the unweighted
    sum of eq. simpleRayleighQuotient."""
    LY = np.column_stack([apply_L(Y[:, i]) for i in range(Y.shape[1])])
    Gram = Y.T @ Y
    G = -(Y.T @ LY)
    G = 0.5 * (G + G.T)
    # generalised symmetric problem G q = mu Gram q (Gram ~ I for orthonormal Y)
    Lc = np.linalg.cholesky(0.5 * (Gram + Gram.T))
    Li = np.linalg.inv(Lc)
    mu, Q = np.linalg.eigh(Li @ G @ Li.T)
    Q = Li.T @ Q
    Z = Y @ Q
    LZ = LY @ Q
    res = np.array([np.linalg.norm(LZ[:, i] + mu[i] * Z[:, i]) / (abs(mu[i]) * np.linalg.norm(Z[:, i]))
                    for i in range(Z.shape[1])])
    return mu, Z, res


@dataclass
class EigsResult:
    mu: np.ndarray              # lambda_h^2 per converged pair
    beta: np.ndarray            # Ritz values of S
    res: np.ndarray             # L_h eigen-residuals ||L z + mu z|| / (mu ||z||)
    Y: np.ndarray               # eigenvectors (unit 2-norm columns)
    wave_solves: int
    restarts: int
    probes: int = 1
    history: List[int] = field(default_factory=list)


def _project_out(Y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """w <- w - Y (Y^T w), one vector at a time (modified Gram-Schmidt)."""
    for i in range(Y.shape[1]):
        w = w - np.dot(w, Y[:, i]) * Y[:, i]
    return w


def krylov_schur_run(apply_S: Op, v: np.ndarray, Y_locked: np.ndarray, m: int, n_keep: int,
                     tol_ritz: float, stop, max_wave_solves: int):
    """One Krylov-Schur run on S deflated by the locked vectors.

    The decomposition kept between restarts is S V_p = V_p T_p + v_{p+1} b^T
    with orthonormal V orthogonal to Y_locked.  Each cycle extends it by
    Arnoldi steps to size m -- every new vector w = S v_j is orthogonalised by
    modified Gram-Schmidt first against the locked vectors, then against
    V (Alg. 3) -- takes the Schur form of the projected matrix (S is symmetric,
    being a function of the symmetric L_h, so this is its symmetric
    eigendecomposition), orders the Ritz values by |theta| descending (the
    "largestAbs" wanted set), and asks ``stop(theta, converged)`` whether to
    end; otherwise it keeps the leading ``n_keep`` Ritz vectors and the
    residual vector.  A Ritz pair is converged when its residual
    |h_{m+1,m} q_{m,i}| <= tol_ritz |theta_i|.

    Returns (theta, Ritz vectors, converged flags, wave_solves, restarts).
    """
    N = v.size
    V = np.zeros((N, m + 1))
    T = np.zeros((m + 1, m))
    v = _project_out(Y_locked, _project_out(Y_locked, v))
    V[:, 0] = v / np.linalg.norm(v)
    p = 0
    wave_solves = 0
    restarts = 0
    while True:
        for j in range(p, m):
            w = apply_S(V[:, j])
            wave_solves += 1
            w = _project_out(Y_locked, w)
            for i in range(j + 1):
                T[i, j] = np.dot(w, V[:, i])
                w = w - T[i, j] * V[:, i]
            T[j + 1, j] = np.linalg.norm(w)
            V[:, j + 1] = w / T[j + 1, j]
        A = 0.5 * (T[:m, :m] + T[:m, :m].T)
        theta, Q = np.linalg.eigh(A)
        order = np.argsort(-np.abs(theta), kind="stable")
        theta = theta[order]
        Q = Q[:, order]
        beta_m = T[m, m - 1]
        conv = np.abs(beta_m * Q[m - 1, :]) <= tol_ritz * np.abs(theta)
        if stop(theta, conv) or wave_solves >= max_wave_solves:
            return theta, V[:, :m] @ Q, conv, wave_solves, restarts
        V[:, :n_keep] = V[:, :m] @ Q[:, :n_keep]
        V[:, n_keep] = V[:, m]
        V[:, n_keep + 1:] = 0.0
        T[:] = 0.0
        T[:n_keep, :n_keep] = np.diag(theta[:n_keep])
        T[n_keep, :n_keep] = beta_m * Q[m - 1, :n_keep]
        p = n_keep
        restarts += 1


def _leading_converged(conv: np.ndarray) -> int:
    n = 0
    while n < conv.size and conv[n]:
        n += 1
    return n


def eigs(apply_S: Op, apply_L: Op, v0: np.ndarray, k: int, m: int, probe_vector,
         tol_ritz: float = 1e-12, tol_res: float = 1e-8, max_wave_solves: int = 100000,
         n_keep: int | None = None, band_rel: float = 1e-10) -> EigsResult:
    """All eigenpairs of S whose |beta| reaches the k-th largest, with multiplicity.

    Run 0 starts from v0 and ends when its leading k Ritz pairs have
    converged; every leading converged pair is locked.  A Krylov space built
    from one vector holds only one direction of each repeated eigenvalue, so
    further runs ("probes") start from fresh vectors ``probe_vector(p)``
    deflated against the locked set.  A probe ends when its leading Ritz pair
    has converged and either lies below the band (|theta_1| < (1 - band_rel)
    theta_k, theta_k the k-th largest locked |beta|) -- then the search is
    complete -- or every leading Ritz value inside the band has converged,
    which are then locked before the next probe.

    Stage 2 is one Rayleigh-Ritz projection of L_h on all locked vectors
    (eq. discreteRayleighQuotient, blockwise), which separates vectors whose
    beta agree to rounding while their mu differ.  Pairs are returned ordered
    by |beta| descending.
    """
    if n_keep is None:
        n_keep = max(k, (m + k) // 2)
    n_keep = min(n_keep, m - 1)
    N = v0.size
    Y = np.zeros((N, 0))
    th_locked = np.zeros(0)
    wave_solves = 0
    restarts = 0
    history = []
    probe = 0
    while True:
        if probe == 0:
            def stop(theta, conv):
                return _leading_converged(conv) >= k
            v = v0
        else:
            theta_k = np.sort(np.abs(th_locked))[::-1][k - 1]
            floor = (1.0 - band_rel) * theta_k

            def stop(theta, conv, floor=floor):
                if not conv[0]:
                    return False
                if abs(theta[0]) < floor:
                    return True
                n_band = int(np.sum(np.abs(theta) >= floor))
                return _leading_converged(conv) >= n_band
            v = probe_vector(probe)
        theta, R, conv, ws, rs = krylov_schur_run(apply_S, v, Y, m, n_keep, tol_ritz, stop,
                                                   max_wave_solves - wave_solves)
        wave_solves += ws
        restarts += rs
        nlead = _leading_converged(conv)
        history.append(nlead)
        if wave_solves >= max_wave_solves and not (probe == 0 and nlead >= k):
            if probe == 0 or nlead == 0:
                raise RuntimeError("eigensolver did not converge within max_wave_solves")
        if probe > 0:
            theta_k = np.sort(np.abs(th_locked))[::-1][k - 1]
            if abs(theta[0]) < (1.0 - band_rel) * theta_k:
                break
            nlead = min(nlead, int(np.sum(np.abs(theta) >= (1.0 - band_rel) * theta_k)))
        Y = np.column_stack([Y, R[:, :nlead]])
        th_locked = np.concatenate([th_locked, theta[:nlead]])
        probe += 1
        if wave_solves >= max_wave_solves:
            break
    mu, Z, res = rayleigh_ritz_L(apply_L, Y)
    coef = Y.T @ Z
    beta = th_locked @ (coef ** 2) / np.sum(coef ** 2, axis=0)
    idx = np.argsort(-np.abs(beta), kind="stable")
    Z = Z[:, idx] / np.linalg.norm(Z[:, idx], axis=0)
    return EigsResult(mu=mu[idx], beta=beta[idx], res=res[idx], Y=Z, wave_solves=wave_solves,
                      restarts=restarts, probes=probe, history=history)
