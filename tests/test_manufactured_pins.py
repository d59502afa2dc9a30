"""Manufactured smooth-coefficient solution through the whole chain that
produces the oracle's inputs and runs its scheme: Q1 assembly with a
cell-wise kappa, load vectors of an analytic source, the CEM-GMsFEM spaces
of Section 3.1, the Galerkin blocks of eq. (3.8), the projected initial
state and the time stepping (fine backward Euler, eq. (2.3), and the
splitting scheme, eqs. (2.4)-(2.5)).

    kappa(x, y) = 1 + 0.5 sin(2 pi x) sin(2 pi y) + 0.5 x,
    u(x, y, t)  = exp(-t) sin(pi x) sin(pi y),
    f           = u_t - div(kappa grad u)
                = exp(-t) [ (2 pi^2 kappa - 1) s - kappa_x s_x - kappa_y s_y ],
with s = sin(pi x) sin(pi y). kappa is not symmetric in x <-> y, so a
transposed cell numbering in the assembly is visible.

Observed orders: about 2 in h (fine backward Euler, L2 at t = T), about 1
in the time step, and an error that falls as H falls at fixed H/h (with the
oversampling layers growing like log(1/H), as the CEM localisation needs).
Two planted mistakes in the fine-grid assembly (a transposed cell
numbering, a wrong mass stencil) break the h-order pin."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle.scheme as S
import problem.fem as FEM
from oracle.finebe import fine_backward_euler
from problem.build import diagnostics, project_blocks
from problem.cem import CoarseGrid, cem_basis, local_spectral, split_spaces

PI = np.pi


def kappa_fn(x, y):
    return 1.0 + 0.5 * np.sin(2 * PI * x) * np.sin(2 * PI * y) + 0.5 * x


def source_fn(x, y):
    """f / exp(-t) for the manufactured solution."""
    s = np.sin(PI * x) * np.sin(PI * y)
    sx = PI * np.cos(PI * x) * np.sin(PI * y)
    sy = PI * np.sin(PI * x) * np.cos(PI * y)
    kx = PI * np.cos(2 * PI * x) * np.sin(2 * PI * y) + 0.5
    ky = PI * np.sin(2 * PI * x) * np.cos(2 * PI * y)
    return (2 * PI ** 2 * kappa_fn(x, y) - 1.0) * s - kx * sx - ky * sy


def u0_fn(x, y):
    return np.sin(PI * x) * np.sin(PI * y)


def fine_grid(n):
    """kappa at the cell centres; cell (iy, ix) is row iy of the array."""
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    return FEM.FineGrid(kappa_fn(X, Y))


def l2(fine, e):
    return float(np.sqrt(e @ (fine.M @ e)))


def fine_be_error(n, dt, T):
    fine = fine_grid(n)
    b = fine.load_smooth(source_fn)
    u0 = fine.nodal(u0_fn)
    steps = int(round(T / dt))
    U = fine_backward_euler(fine.M, fine.A, u0, dt, steps, lambda m: b * np.exp(-(m + 1) * dt))
    exact = u0 * np.exp(-steps * dt)
    return l2(fine, U[-1] - exact) / l2(fine, exact)


def multiscale_error(n_c, layers, dt, T, split=None):
    """Relative L2 error at T of the coarse solution u_H = Psi x.
    split=None: every CEM function in V_H1 (d2 = 0: backward Euler in V_H);
    split=(J1, J2): the eigen-index split of the splitting scheme; dt=None
    then takes half the largest stable step (1 - gamma^2)/lambda2."""
    fine = fine_grid(10 * n_c)
    cg = CoarseGrid(fine, n_c)
    _, _, spsi = local_spectral(cg, 5)
    phis = cem_basis(cg, 5, layers, spsi)
    P1, P2 = split_spaces(cg, phis, 2, 3)
    P1, P2 = P1.toarray(), P2.toarray()
    if split is None:
        P1, P2 = np.hstack([P1, P2]), np.zeros((P1.shape[0], 0))
    bl = project_blocks(fine, sp.csc_matrix(P1), sp.csc_matrix(P2))
    if dt is None:
        dt = 0.5 * diagnostics(bl, with_cond=False)["dt_max"]
    Psi = np.hstack([P1, P2])
    G = Psi.T @ fine.load_smooth(source_fn)
    steps = max(1, int(round(T / dt)))
    blk = S.Blocks(bl["M11"], bl["M12"], bl["M22"], bl["A11"], bl["A12"], bl["A22"], steps * dt, dt, 1)
    src = S.Source(G[:, None], np.exp(-(np.arange(steps) + 1) * dt)[None, None, :], S.TIME_FINE, 1, steps)
    u0 = fine.nodal(u0_fn)
    x0 = np.linalg.solve(blk.M, Psi.T @ (fine.M @ u0))   # L2 projection onto V_H
    X = S.fine_composition(blk, src, x0)
    exact = u0 * np.exp(-steps * dt)
    return l2(fine, Psi @ X[-1] - exact) / l2(fine, exact), dt


def _orders(errs):
    return [float(np.log2(a / b)) for a, b in zip(errs[:-1], errs[1:])]


def check_h_order():
    errs = [fine_be_error(n, 2e-5, 0.02) for n in (10, 20, 40)]
    return errs, _orders(errs)


def test_h_order_is_two():
    errs, orders = check_h_order()
    assert errs[-1] < 1e-3, errs
    assert all(1.8 < q < 2.2 for q in orders), (errs, orders)


def test_dt_order_is_one():
    """h = 1/80 keeps the spatial error (~2e-4) well below the time error."""
    errs = [fine_be_error(80, dt, 1.2) for dt in (0.4, 0.2, 0.1)]
    orders = _orders(errs)
    assert all(0.9 < q < 1.3 for q in orders), (errs, orders)


@pytest.mark.slow
def test_error_falls_with_H():
    """Backward Euler in the CEM-GMsFEM space V_H (J = 5 functions per
    coarse element) at H/h = 10, dt small enough for the spatial error to
    dominate."""
    errs = [multiscale_error(n_c, layers, 1e-3, 0.1)[0] for n_c, layers in ((2, 2), (4, 3), (8, 4))]
    assert errs[0] < 0.03 and errs[-1] < 1e-3, errs
    assert all(a > 2.0 * b for a, b in zip(errs[:-1], errs[1:])), errs


@pytest.mark.slow
def test_splitting_scheme_tracks_the_manufactured_solution():
    """The partially explicit scheme with V_H1 = 2 and V_H2 = 3 CEM functions
    per element, at half its largest stable step, stays within the
    accuracy of backward Euler in the whole space V_H at the same step."""
    e_split, dt = multiscale_error(4, 3, None, 0.05, split=(2, 3))
    e_be, _ = multiscale_error(4, 3, dt, 0.05)
    assert e_split < 5e-3, e_split
    assert abs(e_split - e_be) < 0.25 * e_be, (e_split, e_be)


def test_planted_transposed_kappa_is_caught(monkeypatch):
    """The assembly numbers cells row-major; weighting cell (iy, ix) with
    kappa of cell (ix, iy) leaves an O(1) consistency error."""
    orig = FEM.assemble

    def wrong(conn, n_nodes, cell_k=None, cell_m=None, h=1.0):
        if cell_k is not None:
            n = int(round(np.sqrt(len(cell_k))))
            if n * n == len(cell_k):
                cell_k = np.asarray(cell_k).reshape(n, n).T.ravel()
        return orig(conn, n_nodes, cell_k, cell_m, h)

    monkeypatch.setattr(FEM, "assemble", wrong)
    errs, orders = check_h_order()
    assert not all(1.8 < q < 2.2 for q in orders), (errs, orders)


def test_planted_mass_stencil_is_caught(monkeypatch):
    """A mass stencil whose weights sum to the wrong total (a dropped
    corner coupling) is caught by the same pin."""
    wrong = FEM.ME_REF.copy()
    wrong[0, 2] = wrong[2, 0] = wrong[1, 3] = wrong[3, 1] = 0.0
    monkeypatch.setattr(FEM, "ME_REF", wrong)
    errs, orders = check_h_order()
    assert not (errs[-1] < 1e-3 and all(1.8 < q < 2.2 for q in orders)), (errs, orders)
