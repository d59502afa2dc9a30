"""CEM-GMsFEM multiscale spaces (paper Section 3.1, eqs. (3.1)-(3.3)) and the
split of V_cem into V_H1 and V_H2.

Readings adopted where the paper leaves a choice:
  * weight of the auxiliary inner product: kappa_tilde = kappa * H^-2;
  * the local spectral space V(K_i) is the restriction of H^1_0(Omega):
    natural (Neumann) condition on interior coarse edges, zero on the
    boundary of Omega;
  * the CEM basis phi lives in H^1_0(K_i^+) and the multiplier mu in the
    auxiliary space of the oversampled patch K_i^+;
  * V_H1 = span of the CEM functions built from the J1 lowest local
    eigenfunctions of every coarse element, V_H2 = span of those built from
    eigenfunctions J1+1..J1+J2 (one construction with J = J1 + J2);
  * every basis column is normalised to unit L2(Omega) norm (this rescales
    coefficients only; the spaces are unchanged).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import KE_REF, ME_REF, cell_connectivity


class CoarseGrid:
    def __init__(self, fine, n_c):
        self.fine = fine
        self.n_c = n_c
        assert fine.n % n_c == 0
        self.m = fine.n // n_c          # fine cells per coarse element side
        self.H = 1.0 / n_c
        self.n_elem = n_c * n_c

    def element_nodes(self, e):
        """Full-grid node ids of coarse element e (row-major local order)."""
        n, m = self.fine.n, self.m
        ey, ex = divmod(e, self.n_c)
        ly, lx = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
        return ((ey * m + ly) * (n + 1) + ex * m + lx).ravel()

    def element_cells(self, e):
        n, m = self.fine.n, self.m
        ey, ex = divmod(e, self.n_c)
        ly, lx = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        return ((ey * m + ly) * n + ex * m + lx).ravel()

    def patch(self, e, layers):
        """Oversampled patch K_e^+ = K_e plus `layers` coarse layers, clipped to
        the domain. Returns (element ids in the patch, full node ids of the
        nodes strictly inside the patch rectangle)."""
        n, m, n_c = self.fine.n, self.m, self.n_c
        ey, ex = divmod(e, n_c)
        y0, y1 = max(ey - layers, 0), min(ey + layers, n_c - 1)
        x0, x1 = max(ex - layers, 0), min(ex + layers, n_c - 1)
        elems = np.array([yy * n_c + xx for yy in range(y0, y1 + 1) for xx in range(x0, x1 + 1)])
        iy = np.arange(y0 * m + 1, (y1 + 1) * m)
        ix = np.arange(x0 * m + 1, (x1 + 1) * m)
        IY, IX = np.meshgrid(iy, ix, indexing="ij")
        return elems, (IY * (n + 1) + IX).ravel()


def local_spectral(cg, J):
    """Local generalized eigenproblems, eq. (3.1): on every coarse element
    A_e psi = lambda S_e psi, with A_e the kappa-weighted Q1 stiffness and
    S_e the (kappa H^-2)-weighted Q1 mass over the element's cells, zero
    values on the boundary of Omega. Returns per element the J lowest
    eigenvalues, the S_e-orthonormal eigenvectors on the element's local
    nodes, and S_e @ eigenvectors (used by the constraints of eq. (3.2))."""
    fine = cg.fine
    m, h = cg.m, fine.h
    nl = (m + 1) ** 2
    conn = cell_connectivity(m, m)
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    flat = rows * nl + cols
    kref = np.tile(KE_REF.ravel(), m * m)
    mref = np.tile(ME_REF.ravel(), m * m) * h * h
    kap = fine.kappa.ravel()
    boundary = np.ones(fine.n_nodes, dtype=bool)
    boundary[fine.interior] = False
    lam = np.zeros((cg.n_elem, J))
    psi = np.zeros((cg.n_elem, nl, J))
    spsi = np.zeros((cg.n_elem, nl, J))
    for e in range(cg.n_elem):
        kc = np.repeat(kap[cg.element_cells(e)], 16)
        A = np.bincount(flat, weights=kc * kref, minlength=nl * nl).reshape(nl, nl)
        S = np.bincount(flat, weights=kc * mref / cg.H ** 2, minlength=nl * nl).reshape(nl, nl)
        free = ~boundary[cg.element_nodes(e)]
        Af = A[np.ix_(free, free)]
        Sf = S[np.ix_(free, free)]
        w, v = sla.eigh(Af, Sf, subset_by_index=[0, J - 1])
        lam[e] = w
        psi[e][free] = v
        spsi[e] = S @ psi[e]
    return lam, psi, spsi


def cem_basis(cg, J, layers, spsi, return_checks=False):
    """Constraint energy minimising basis, eq. (3.2): for every element i and
    j < J find phi in H^1_0(K_i^+) and multipliers mu with
        a(phi, v) + s(mu, v) = 0  for all v,
        s(phi, nu) = s(psi_j^(i), nu)  for all nu in V_aux(K_i^+).
    Discretely [A+ C^T; C 0][phi; mu] = [0; e_(i,j)], solved for the J
    right-hand sides of element i with one sparse LU of the saddle-point
    matrix of the patch. Returns a list (per element) of (full-grid node ids
    of the patch interior, (n_free, J) array of phi), and optionally the
    constraint residuals."""
    fine = cg.fine
    Kfull = fine.K_full.tocsr()
    n_nodes = fine.n_nodes
    lookup = -np.ones(n_nodes, dtype=np.int64)
    out, checks = [], []
    for i in range(cg.n_elem):
        elems, free_ids = cg.patch(i, layers)
        nf = free_ids.size
        lookup[free_ids] = np.arange(nf)
        Ap = Kfull[free_ids][:, free_ids]
        rows, cols, vals = [], [], []
        for a, k in enumerate(elems):
            loc = lookup[cg.element_nodes(k)]
            keep = loc >= 0
            for j in range(J):
                rows.append(np.full(int(keep.sum()), a * J + j))
                cols.append(loc[keep])
                vals.append(spsi[k][keep, j])
        n_aux = elems.size * J
        C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n_aux, nf))
        lu = spla.splu(sp.bmat([[Ap, C.T], [C, None]], format="csc"), permc_spec="MMD_AT_PLUS_A",
                       diag_pivot_thresh=0.01, options=dict(SymmetricMode=True))
        a_i = int(np.flatnonzero(elems == i)[0])
        rhs = np.zeros((nf + n_aux, J))
        rhs[nf + a_i * J + np.arange(J), np.arange(J)] = 1.0
        phi = lu.solve(rhs)[:nf]
        out.append((free_ids.copy(), phi))
        if return_checks:
            E = np.zeros((n_aux, J))
            E[a_i * J:(a_i + 1) * J, :] = np.eye(J)
            checks.append(np.abs(C @ phi - E).max())
        lookup[free_ids] = -1
    return (out, checks) if return_checks else out


def split_spaces(cg, phis, J1, J2):
    """Assemble Psi1 (n_dof x d1) and Psi2 (n_dof x d2), columns ordered
    element-major (element i, eigen-index j), each column scaled to unit
    L2 norm on the fine grid."""
    fine = cg.fine
    M = fine.M
    cols = {1: ([], [], []), 2: ([], [], [])}
    counts = {1: 0, 2: 0}
    for i, (ids, phi) in enumerate(phis):
        dofs = fine.node2dof[ids]
        assert (dofs >= 0).all()
        for j in range(J1 + J2):
            which = 1 if j < J1 else 2
            r, c, v = cols[which]
            r.append(dofs)
            c.append(np.full(dofs.size, counts[which]))
            v.append(phi[:, j])
            counts[which] += 1
    mats = []
    for which in (1, 2):
        r, c, v = cols[which]
        P = sp.csc_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))),
                          shape=(fine.n_dof, counts[which]))
        norms = np.sqrt(np.asarray(P.multiply(M @ P).sum(axis=0)).ravel())
        mats.append((P @ sp.diags(1.0 / norms)).tocsc())
    return mats[0], mats[1]
