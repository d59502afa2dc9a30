"""Pins for the oracle's discrete adjoint: the dot-product identity of the
linear map (x0, H) -> X, central finite differences of a quadratic loss
(exact up to rounding), and the transpose of a single fine propagator
against its explicitly formed matrix."""
import numpy as np
import pytest

import oracle.adjoint as ADJ
import oracle.scheme as S
from problem import build_problem


@pytest.mark.parametrize("name", ["t0", "t1", "t2"])
def test_dot_product_identity(name):
    p = build_problem(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    rng = np.random.default_rng(11)
    x0 = rng.standard_normal(bl.D)
    H = rng.standard_normal(p["H"].shape[1:])
    Xbar = rng.standard_normal((bl.N + 1, bl.D))
    X = ADJ.forward_linear(bl, p["G"], p["time_mode"], x0, H)
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, lam = ADJ.adjoint(bl, sbar, Xbar)
    lhs = np.sum(X * Xbar)
    rhs = np.sum(x0 * x0b) + np.sum(H * Hb)
    assert abs(lhs - rhs) <= 1e-11 * (np.abs(X * Xbar).sum() + np.abs(x0 * x0b).sum() + np.abs(H * Hb).sum())


def test_fine_propagator_transpose_matches_matrix():
    """F_hom as an explicit matrix (columns = F_hom of unit vectors) and its
    transpose applied to a vector equals the adjoint sweep."""
    p = build_problem("t0")
    bl = S.Blocks.from_problem(p)
    zero = S.Source(None, None, S.TIME_FINE, bl.N, bl.P)
    Phi = np.stack([S.fine_propagator(bl, zero, e, 0) for e in np.eye(bl.D)], axis=1)
    lam = np.random.default_rng(3).standard_normal(bl.D)
    back, _ = ADJ.fine_propagator_adjoint(bl, lam)
    np.testing.assert_allclose(back, Phi.T @ lam, rtol=1e-10, atol=1e-12 * np.abs(Phi.T @ lam).max())


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_finite_differences_quadratic_loss(name):
    """L = 1/2 |X_N - ref|_M^2 + 1/2 sum_n dt |X_n - ref_n|_M^2 is quadratic
    in (x0, H): central differences have no truncation error."""
    p = build_problem(name)
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(5)
    scale = 1e-3
    x0 = scale * rng.standard_normal(bl.D)
    H = rng.standard_normal(p["H"].shape[1:])
    ref = ADJ.forward_linear(bl, p["G"], p["time_mode"], 0 * x0, H + 0.3 * rng.standard_normal(H.shape))
    M = bl.M

    def loss(X):
        e = X - ref
        q = np.einsum("nd,de,ne->n", e, M, e)
        return 0.5 * q[-1] + 0.5 * bl.dt * q.sum()

    X = ADJ.forward_linear(bl, p["G"], p["time_mode"], x0, H)
    e = X - ref
    Xbar = (bl.dt * e) @ M
    Xbar[-1] += e[-1] @ M
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, _ = ADJ.adjoint(bl, sbar, Xbar)
    dirs = []
    for _ in range(4):
        dx, dH = rng.standard_normal(bl.D), rng.standard_normal(H.shape)
        nrm = np.sqrt(np.sum(dx ** 2) + np.sum(dH ** 2))
        dirs.append((dx / nrm, dH / nrm))
    for i in range(3):  # coordinate directions of H
        dH = np.zeros(H.shape)
        dH.flat[rng.integers(H.size)] = 1.0
        dirs.append((np.zeros(bl.D), dH))
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, x0b, Hb, dirs, h=1e-3)
    np.testing.assert_allclose(fd, ad, rtol=1e-6, atol=1e-9 * np.abs(ad).max())
