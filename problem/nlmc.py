"""NLMC split of the multiscale space for channelised media (paper Section 3.2,
eqs. (3.4)-(3.7)): one constraint energy minimising basis function per
connected high-contrast piece ("fracture") of every coarse block and one per
block's matrix region; V_H1 holds the fracture functions made s-orthogonal to
their mean, V_H2 the matrix functions and the mean.

Readings adopted where the paper leaves a choice:
  * a fracture of coarse block K_i is a connected component (through shared
    cell edges, inside K_i) of the cells with kappa >= kappa_threshold; the
    matrix region K_{i,m} is the rest of K_i;
  * the constraints of eq. (3.6) are exact integrals of the Q1 basis
    functions over the region's cells (h^2/4 per cell corner);
  * psi_bar of eq. (3.7) sums every basis function (matrix and fracture) and
    divides by L = the number of fracture functions (the printed
    L = sum_{i=1}^N m_i); the s-orthogonalisation against psi_bar uses
    s(u, v) = int kappa H^-2 u v, as for the auxiliary spaces of Section 3.1;
  * V_H1 = the first L - 1 orthogonalised fracture functions (element-major
    order), V_H2 = [psi_bar, psi_0^(1..N_e)] (variant "paper"); with this
    V_H2 the largest Rayleigh quotient lambda2 grows with the contrast on our
    channel media (psi_bar carries the fracture functions' gradients inside
    the channels), so a second variant "fm" splits the same NLMC space by
    continuum only: V_H1 = every fracture function, V_H2 = the matrix
    functions (lambda2, gamma and the stable step then do not depend on the
    contrast);
  * every basis column is normalised to unit L2(Omega) norm (coefficients
    only; the spaces are unchanged).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

REFINE_STEPS = 5  # iterative refinement of every patch's saddle-point solve


def fracture_regions(cg, threshold):
    """Per coarse element: (matrix cells, [cells of each fracture]) as
    full-grid cell ids; fractures ordered by their smallest cell id."""
    fine = cg.fine
    n, m = fine.n, cg.m
    high = fine.kappa.ravel() >= threshold
    out = []
    for e in range(cg.n_elem):
        cells = cg.element_cells(e)
        hi = cells[high[cells]]
        lab = {}
        comps = []
        for c in sorted(hi.tolist()):
            if c in lab:
                continue
            stack, comp = [c], []
            lab[c] = len(comps)
            while stack:
                x = stack.pop()
                comp.append(x)
                cy, cx = divmod(x, n)
                for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    yy, xx = cy + dy, cx + dx
                    if not (0 <= yy < n and 0 <= xx < n):
                        continue
                    nb = yy * n + xx
                    if nb in lab or not high[nb]:
                        continue
                    ey, ex = divmod(e, cg.n_c)
                    if not (ey * m <= yy < (ey + 1) * m and ex * m <= xx < (ex + 1) * m):
                        continue
                    lab[nb] = lab[c]
                    stack.append(nb)
            comps.append(np.array(sorted(comp)))
        out.append((cells[~high[cells]], comps))
    return out


def _region_row(fine, cells, lookup):
    """Integrals of the free Q1 basis functions over `cells` (h^2/4 per
    corner): (column ids in the patch, values)."""
    n = fine.n
    cy, cx = np.divmod(cells, n)
    corners = np.concatenate([cy * (n + 1) + cx, cy * (n + 1) + cx + 1,
                              (cy + 1) * (n + 1) + cx, (cy + 1) * (n + 1) + cx + 1])
    loc = lookup[corners]
    keep = loc >= 0
    vals = np.full(int(keep.sum()), fine.h * fine.h / 4.0)
    return loc[keep], vals


def nlmc_basis(cg, regions, layers, return_checks=False):
    """Eq. (3.6) on every oversampled patch: find psi in H^1_0(K_i^+) and
    multipliers with a(psi, v) + sum_regions mu_r int_r v = 0 for all v and
    int_r psi = delta (r the region of psi, every region of every block in
    K_i^+), one sparse LU of the saddle-point matrix per patch. Returns per
    element (full-grid node ids of the patch interior, (n_free, 1 + m_i)
    array: the matrix function then the fracture functions)."""
    fine = cg.fine
    Kfull = fine.K_full.tocsr()
    lookup = -np.ones(fine.n_nodes, dtype=np.int64)
    out, checks = [], []
    for i in range(cg.n_elem):
        elems, free_ids = cg.patch(i, layers)
        nf = free_ids.size
        lookup[free_ids] = np.arange(nf)
        Ap = Kfull[free_ids][:, free_ids]
        rows, cols, vals = [], [], []
        own = None
        r = 0
        for k in elems:
            mat, fr = regions[k]
            if k == i:
                own = r
            for cells in [mat] + fr:
                c, v = _region_row(fine, cells, lookup)
                rows.append(np.full(c.size, r))
                cols.append(c)
                vals.append(v)
                r += 1
        C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(r, nf))
        K = sp.bmat([[Ap, C.T], [C, None]], format="csc")
        lu = spla.splu(K, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.01, options=dict(SymmetricMode=True))
        nb = 1 + len(regions[i][1])
        rhs = np.zeros((nf + r, nb))
        rhs[nf + own + np.arange(nb), np.arange(nb)] = 1.0
        # the fracture rows of the stiffness carry the contrast, and the LU
        # with threshold pivoting leaves the constraints of eq. (3.6) violated
        # by up to ~1e-5 at contrast 1e6: iterative refinement with the same
        # factors brings them to rounding level
        x = lu.solve(rhs)
        for _ in range(REFINE_STEPS):
            x += lu.solve(rhs - K @ x)
        psi = x[:nf]
        out.append((free_ids.copy(), psi))
        if return_checks:
            E = np.zeros((r, nb))
            E[own:own + nb] = np.eye(nb)
            checks.append(np.abs(C @ psi - E).max())
        lookup[free_ids] = -1
    return (out, checks) if return_checks else out


def region_data(cg, regions, J=None):
    """Constraint data of eq. (3.6) per coarse element for the GPU set-up
    pipeline: counts[k] = 1 + number of fractures of element k, and
    rdata (n_el x (m+1)^2 x J): slot l of element k (0: matrix region,
    1..: fractures) on the element's local node (row-major) holds the region's
    integral of that node's Q1 function, h^2/4 per region cell the node is a
    corner of."""
    fine = cg.fine
    n, m, n_c = fine.n, cg.m, cg.n_c
    counts = np.array([1 + len(fr) for _, fr in regions], dtype=np.int32)
    J = int(counts.max()) if J is None else int(J)
    ml = m + 1
    rdata = np.zeros((cg.n_elem, ml * ml, J))
    q = fine.h * fine.h / 4.0
    for k, (mat, fr) in enumerate(regions):
        ey, ex = divmod(k, n_c)
        for l, cells in enumerate([mat] + list(fr)):
            cy, cx = np.divmod(np.asarray(cells), n)
            ly, lx = cy - ey * m, cx - ex * m
            for dy in (0, 1):
                for dx in (0, 1):
                    np.add.at(rdata[k, :, l], (ly + dy) * ml + (lx + dx), q)
    return counts, rdata


def nlmc_split(cg, psis, variant="paper"):
    """Psi1 and Psi2 from the NLMC functions. variant "paper": Section 3.2 as
    printed, Psi1 (n_dof x (L-1)) the s-orthogonalised fracture functions
    less the last, Psi2 (n_dof x (N_e + 1)) = [psi_bar, matrix functions].
    variant "fm": Psi1 = every fracture function, Psi2 = the matrix
    functions (the same NLMC space, split by continuum only)."""
    fine = cg.fine
    nd = fine.n_dof

    def column(ids, v):
        x = np.zeros(nd)
        dofs = fine.node2dof[ids]
        assert (dofs >= 0).all()
        x[dofs] = v
        return x

    mats = [column(ids, psi[:, 0]) for ids, psi in psis]
    fracs = [column(ids, psi[:, m]) for ids, psi in psis for m in range(1, psi.shape[1])]
    L = len(fracs)
    M = fine.M

    def normed(cols):
        P = np.stack(cols, axis=1)
        nrm = np.sqrt(np.einsum("ij,ij->j", P, M @ P))
        return sp.csc_matrix(P / nrm)

    if variant == "fm":
        if L < 1:
            raise ValueError("the NLMC split needs at least one fracture function")
        return normed(fracs), normed(mats)
    if variant != "paper":
        raise ValueError(variant)
    if L < 2:
        raise ValueError("the NLMC split needs at least two fracture functions")
    bar = (np.sum(mats, axis=0) + np.sum(fracs, axis=0)) / L
    Sb = s_matrix(cg) @ bar
    sbb = float(bar @ Sb)
    tilde = [f - float(f @ Sb) / sbb * bar for f in fracs]
    return normed(tilde[:L - 1]), normed([bar] + mats)


def s_matrix(cg):
    """s(u, v) = int kappa H^-2 u v on the interior unknowns (Q1 mass with
    cell weights kappa H^-2)."""
    from .fem import assemble
    fine = cg.fine
    _, Ms = assemble(fine.conn, fine.n_nodes, None, fine.kappa.ravel() / cg.H ** 2, fine.h)
    return Ms[fine.interior][:, fine.interior].tocsr()
