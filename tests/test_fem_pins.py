"""Pins for the fine-grid FEM and the CEM-GMsFEM construction (inputs of the
path): element matrices against quadrature, an exact discrete eigenvector,
closed-form local eigenvalues, and the CEM constraints of eq. (3.2)."""
import numpy as np
import pytest
import scipy.linalg as sla

from problem import build_problem, build_spaces
from problem.cem import CoarseGrid, cem_basis, local_spectral
from problem.fem import KE_REF, ME_REF, FineGrid


def _q1_by_quadrature(h):
    """Element matrices of the bilinear square element by 2x2 Gauss
    quadrature of the shape functions (independent of the closed forms)."""
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    nodes = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=float)
    K = np.zeros((4, 4))
    M = np.zeros((4, 4))
    for xi in (0.5 + 0.5 * g):
        for eta in (0.5 + 0.5 * g):
            N = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
            dN = np.array([[-(1 - eta), -(1 - xi)], [1 - eta, -xi], [eta, xi], [-eta, 1 - xi]]) / h
            w = 0.25 * h * h
            K += w * dN @ dN.T
            M += w * np.outer(N, N)
    return K, M


def test_element_matrices_match_quadrature():
    for h in (0.1, 0.025):
        K, M = _q1_by_quadrature(h)
        np.testing.assert_allclose(KE_REF, K, rtol=0, atol=1e-14)
        np.testing.assert_allclose(ME_REF * h * h, M, rtol=0, atol=1e-16)
    assert np.abs(KE_REF.sum(axis=1)).max() < 1e-15
    assert abs(ME_REF.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("n", [8, 20])
def test_discrete_sine_is_exact_eigenvector(n):
    """kappa = 1: the nodal sin(pi x) sin(pi y) satisfies A s = lam_h M s with
    lam_h = 12 (1 - cos(pi h)) / (h^2 (2 + cos(pi h)))."""
    fine = FineGrid(np.ones((n, n)))
    s = fine.nodal(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))
    h = 1.0 / n
    lam = 12 * (1 - np.cos(np.pi * h)) / (h * h * (2 + np.cos(np.pi * h)))
    np.testing.assert_allclose(fine.A @ s, lam * (fine.M @ s), rtol=0, atol=1e-11 * lam * np.abs(fine.M @ s).max())


def test_local_spectral_closed_form():
    """Constant kappa, interior coarse element (Neumann on its edges): the
    eigenvalues of eq. (3.1) with kappa_tilde = kappa H^-2 are
    H^2 (mu_i + mu_j), mu_k = 6 (1 - cos(k pi/m)) / (h^2 (2 + cos(k pi/m)))
    (tensor product of the 1D Neumann Q1 pencil), independent of kappa."""
    n, n_c = 30, 3
    fine = FineGrid(7.5 * np.ones((n, n)))
    cg = CoarseGrid(fine, n_c)
    lam, psi, spsi = local_spectral(cg, 6)
    m, h, H = cg.m, fine.h, cg.H
    th = np.arange(m + 1) * np.pi / m
    mu = 6 * (1 - np.cos(th)) / (h * h * (2 + np.cos(th)))
    ref = np.sort((mu[:, None] + mu[None, :]).ravel())[:6] * H * H
    centre = 4  # the interior element of a 3 x 3 coarse grid
    np.testing.assert_allclose(lam[centre], ref, rtol=1e-10, atol=1e-10)
    # continuum limit pi^2 (i^2 + j^2): 0, pi^2, pi^2, 2 pi^2, 4 pi^2, 4 pi^2
    np.testing.assert_allclose(lam[centre][1:5], np.pi ** 2 * np.array([1, 1, 2, 4]), rtol=0.05)


def test_cem_constraints_and_energy_minimality():
    cfg = dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1,
               contrast=1e4, seed=5)
    from problem.build import make_medium
    fine = FineGrid(make_medium(cfg))
    cg = CoarseGrid(fine, 3)
    lam, psi, spsi = local_spectral(cg, 5)
    phis, checks = cem_basis(cg, 5, 1, spsi, return_checks=True)
    assert max(checks) < 1e-10
    # support inside the oversampled patch, zero on its boundary: ids are
    # strictly interior nodes of the patch rectangle
    for i, (ids, phi) in enumerate(phis):
        elems, free_ids = cg.patch(i, 1)
        assert set(ids.tolist()) == set(free_ids.tolist())
    # energy minimality: perturbations that keep every constraint raise the
    # energy (checked for one element with random null-space directions)
    i = 4
    ids, phi = phis[i]
    elems, _ = cg.patch(i, 1)
    lookup = -np.ones(fine.n_nodes, dtype=int)
    lookup[ids] = np.arange(ids.size)
    C = np.zeros((elems.size * 5, ids.size))
    for a, k in enumerate(elems):
        loc = lookup[cg.element_nodes(k)]
        keep = loc >= 0
        C[a * 5:(a + 1) * 5, loc[keep]] = spsi[k][keep].T
    Ap = fine.K_full[ids][:, ids].toarray()
    Z = sla.null_space(C)
    rng = np.random.default_rng(0)
    for j in range(5):
        e0 = phi[:, j] @ Ap @ phi[:, j]
        for _ in range(3):
            d = Z @ rng.standard_normal(Z.shape[1])
            d *= 1e-3 * np.linalg.norm(phi[:, j]) / np.linalg.norm(d)
            assert (phi[:, j] + d) @ Ap @ (phi[:, j] + d) > e0
            # first-order optimality: a(phi, d) = 0 for constraint-preserving d
            assert abs(phi[:, j] @ Ap @ d) < 1e-8 * e0


def test_blocks_symmetric_spd():
    p = build_problem("t0")
    for k in ("M11", "M22", "A11", "A22"):
        X = p[k]
        np.testing.assert_allclose(X, X.T, atol=0)
        assert np.linalg.eigvalsh(X).min() > 0
    M = np.block([[p["M11"], p["M12"]], [p["M12"].T, p["M22"]]])
    assert np.linalg.eigvalsh(M).min() > 0
    assert p["d1"] == 2 * 4 and p["d2"] == 3 * 4


def test_blocks_equal_fine_grid_forms():
    """Blocks are the fine-grid forms restricted to V_H: for random
    coefficient vectors a, b: a^T M b = (Psi a)^T M_f (Psi b)."""
    p = build_problem("t0", use_cache=False, keep_spaces=True)
    fine, P1, P2 = p["fine"], p["Psi1"], p["Psi2"]
    rng = np.random.default_rng(1)
    a1, a2 = rng.standard_normal(p["d1"]), rng.standard_normal(p["d2"])
    b1, b2 = rng.standard_normal(p["d1"]), rng.standard_normal(p["d2"])
    ua, ub = P1 @ a1 + P2 @ a2, P1 @ b1 + P2 @ b2
    M = np.block([[p["M11"], p["M12"]], [p["M12"].T, p["M22"]]])
    A = np.block([[p["A11"], p["A12"]], [p["A12"].T, p["A22"]]])
    a, b = np.concatenate([a1, a2]), np.concatenate([b1, b2])
    assert abs(a @ M @ b - ua @ fine.M @ ub) < 1e-12 * np.sqrt((ua @ fine.M @ ua) * (ub @ fine.M @ ub))
    assert abs(a @ A @ b - ua @ fine.A @ ub) < 1e-10 * np.sqrt((ua @ fine.A @ ua) * (ub @ fine.A @ ub))
    # unit L2 columns
    np.testing.assert_allclose(np.diag(p["M11"]), 1.0, rtol=1e-12)
    np.testing.assert_allclose(np.diag(p["M22"]), 1.0, rtol=1e-12)
