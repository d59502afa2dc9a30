"""Pins of the quantities every parity verdict and every horizon rests on,
each computed a second way on the fine grid:

* the relative error metric rel_l2_M (mass norm over all coarse-boundary
  states) against the fine-grid L2 norms of the prolonged functions
  u_H = Psi x (the error of Section 5 measured in L2(Omega));
* lambda2 = sup over V_H2 of |v|_a^2 / |v|^2 (the stability condition of
  Section 3.2) against the largest eigenvalue of the fine stiffness on an
  L2-orthonormal basis of the prolonged V_H2;
* gamma^2 of eq. (4.15) (squared cosine between V_H1 and V_H2 in L2) from
  the block formula (the problem generator's diagnostics and the oracle's
  waveform-relaxation module) against the smallest principal angle of the
  prolonged spaces in the L2 inner product.

Each pin is also run on an implementation with a planted mistake, which it
must reject."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle.scheme as S
import oracle.wr as WR
from problem import build_problem
from problem.build import diagnostics


@pytest.fixture(scope="module")
def spaces():
    p = build_problem("t1", use_cache=False, keep_spaces=True)
    P1 = np.asarray(p["Psi1"].todense()) if hasattr(p["Psi1"], "todense") else np.asarray(p["Psi1"])
    P2 = np.asarray(p["Psi2"].todense()) if hasattr(p["Psi2"], "todense") else np.asarray(p["Psi2"])
    Mf = p["fine"].M.toarray()
    Af = p["fine"].A.toarray()
    return p, P1, P2, Mf, Af


def fine_rel_l2(P, Mf, X, Xref):
    """sqrt(sum_n |u_H(X_n) - u_H(Xref_n)|^2_L2 / sum_n |u_H(Xref_n)|^2_L2)
    with u_H = Psi x prolonged to the fine grid."""
    E = P @ (X - Xref).T
    R = P @ Xref.T
    return float(np.sqrt(np.einsum("ij,ik,kj->", E, Mf, E) / np.einsum("ij,ik,kj->", R, Mf, R)))


def check_rel_l2(fn, p, P, Mf, rng):
    bl = S.Blocks.from_problem(p)
    worst = 0.0
    for scale in (1e-6, 0.3, 2.0):
        Xref = rng.standard_normal((bl.N + 1, bl.D))
        X = Xref + scale * rng.standard_normal(Xref.shape)
        want = fine_rel_l2(P, Mf, X, Xref)
        worst = max(worst, abs(fn(bl, X, Xref) - want) / want)
    # closed forms: equal inputs give 0, X = 2 Xref gives 1
    worst = max(worst, abs(fn(bl, Xref, Xref)), abs(fn(bl, 2.0 * Xref, Xref) - 1.0))
    return worst


def test_rel_l2_M_is_the_fine_l2_error(spaces):
    p, P1, P2, Mf, _ = spaces
    P = np.hstack([P1, P2])
    assert check_rel_l2(S.rel_l2_M, p, P, Mf, np.random.default_rng(0)) < 1e-10


def _rel_no_sqrt(bl, X, Xref):
    num = sum(S.m_norm(bl, X[n] - Xref[n]) ** 2 for n in range(X.shape[0]))
    den = sum(S.m_norm(bl, Xref[n]) ** 2 for n in range(X.shape[0]))
    return num / den


def _rel_wrong_denominator(bl, X, Xref):
    num = sum(S.m_norm(bl, X[n] - Xref[n]) ** 2 for n in range(X.shape[0]))
    den = sum(S.m_norm(bl, X[n]) ** 2 for n in range(X.shape[0]))
    return float(np.sqrt(num / den))


def _rel_euclidean(bl, X, Xref):
    return float(np.linalg.norm(X - Xref) / np.linalg.norm(Xref))


def _rel_no_coupling(bl, X, Xref):
    """mass norm without the M12 block"""
    Md = sla.block_diag(bl.M11, bl.M22)
    q = lambda E: float(np.einsum("ij,jk,ik->", E, Md, E))
    return float(np.sqrt(q(X - Xref) / q(Xref)))


@pytest.mark.parametrize("planted", [_rel_no_sqrt, _rel_wrong_denominator, _rel_euclidean, _rel_no_coupling])
def test_planted_rel_l2_mistakes_are_caught(spaces, planted):
    p, P1, P2, Mf, _ = spaces
    P = np.hstack([P1, P2])
    assert check_rel_l2(planted, p, P, Mf, np.random.default_rng(0)) > 1e-3


def fine_lambda2(P2, Mf, Af):
    """largest |v|_a^2/|v|^2 over span(Psi2): fine stiffness on an
    L2-orthonormal basis Q = Psi2 R^-T (R R^T = Psi2^T Mf Psi2), standard
    symmetric eigenvalues."""
    R = np.linalg.cholesky(P2.T @ Mf @ P2)
    Q = sla.solve_triangular(R, P2.T, lower=True).T
    return float(np.linalg.eigvalsh(Q.T @ Af @ Q)[-1])


def fine_gamma2(P1, P2, Mf):
    """cos^2 of the smallest principal angle between span(Psi1) and
    span(Psi2) in the L2 inner product (Mf = L L^T: angles of L^T Psi)."""
    L = np.linalg.cholesky(Mf)
    ang = sla.subspace_angles(L.T @ P1, L.T @ P2)
    return float(np.cos(ang.min()) ** 2)


def check_diagnostics(fn, p, P1, P2, Mf, Af):
    d = fn(p)
    lam, g2 = fine_lambda2(P2, Mf, Af), fine_gamma2(P1, P2, Mf)
    return max(abs(d["lambda2"] - lam) / lam, abs(d["gamma2"] - g2) / g2,
               abs(d["dt_max"] - (1 - g2) / lam) / ((1 - g2) / lam))


def _diag(p):
    return diagnostics({k: p[k] for k in ("M11", "M12", "M22", "A11", "A12", "A22")}, with_cond=False)


def test_lambda2_gamma2_dt_max(spaces):
    p, P1, P2, Mf, Af = spaces
    g2 = fine_gamma2(P1, P2, Mf)
    assert 0.0 < g2 < 1.0
    assert check_diagnostics(_diag, p, P1, P2, Mf, Af) < 1e-9


def test_oracle_gamma_sq_is_the_principal_angle(spaces):
    p, P1, P2, Mf, _ = spaces
    g2 = WR.gamma_sq(S.Blocks.from_problem(p))
    assert abs(g2 - fine_gamma2(P1, P2, Mf)) < 1e-9 * g2


def _diag_no_mass_in_lambda(p):
    d = _diag(p)
    d["lambda2"] = float(np.linalg.eigvalsh(p["A22"])[-1])
    d["dt_max"] = (1 - d["gamma2"]) / d["lambda2"]
    return d


def _diag_wrong_block(p):
    d = _diag(p)
    d["lambda2"] = float(sla.eigh(p["A11"], p["M11"], eigvals_only=True)[-1])
    d["dt_max"] = (1 - d["gamma2"]) / d["lambda2"]
    return d


def _diag_gamma_without_M22(p):
    d = _diag(p)
    X = sla.solve(p["M11"], p["M12"], assume_a="pos")
    d["gamma2"] = float(np.linalg.eigvalsh(p["M12"].T @ X)[-1])
    d["dt_max"] = (1 - d["gamma2"]) / d["lambda2"]
    return d


def _diag_gamma_not_squared(p):
    d = _diag(p)
    d["gamma2"] = float(np.sqrt(d["gamma2"]))
    d["dt_max"] = (1 - d["gamma2"]) / d["lambda2"]
    return d


@pytest.mark.parametrize("planted", [_diag_no_mass_in_lambda, _diag_wrong_block, _diag_gamma_without_M22,
                                     _diag_gamma_not_squared])
def test_planted_diagnostic_mistakes_are_caught(spaces, planted):
    p, P1, P2, Mf, Af = spaces
    assert check_diagnostics(planted, p, P1, P2, Mf, Af) > 1e-3
