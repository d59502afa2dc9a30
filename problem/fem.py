"""Q1 finite elements on the unit square (paper Section 2, the fine-grid
discretisation behind the projected blocks of Section 3.2, eq. (3.8)).

The fine grid has n x n square cells of side h = 1/n. Nodes are numbered
row-major, node (ix, iy) -> iy*(n+1) + ix. Unknowns are the interior nodes
(u = 0 on the boundary, eq. (2.1)); interior node (ix, iy) with
1 <= ix, iy <= n-1 has unknown index (iy-1)*(n-1) + (ix-1).

Element matrices of a square bilinear element with nodes ordered
counter-clockwise (0,0), (1,0), (1,1), (0,1):
  stiffness  kappa/6  * [[4,-1,-2,-1],[-1,4,-1,-2],[-2,-1,4,-1],[-1,-2,-1,4]]
  mass       h^2/36   * [[4,2,1,2],[2,4,2,1],[1,2,4,2],[2,1,2,4]]
(the stiffness of a square Q1 element does not depend on h in 2D).
"""
import numpy as np
import scipy.sparse as sp

KE_REF = np.array([[4, -1, -2, -1],
                   [-1, 4, -1, -2],
                   [-2, -1, 4, -1],
                   [-1, -2, -1, 4]], dtype=np.float64) / 6.0
ME_REF = np.array([[4, 2, 1, 2],
                   [2, 4, 2, 1],
                   [1, 2, 4, 2],
                   [2, 1, 2, 4]], dtype=np.float64) / 36.0


def cell_connectivity(nx, ny, stride=None):
    """Node ids (counter-clockwise) of the nx*ny cells of a structured block
    whose nodes are numbered iy*stride + ix (stride defaults to nx+1).
    Returns an (ny*nx, 4) int array, cells row-major (iy, ix)."""
    if stride is None:
        stride = nx + 1
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    n0 = (iy * stride + ix).ravel()
    return np.stack([n0, n0 + 1, n0 + stride + 1, n0 + stride], axis=1)


def assemble(conn, n_nodes, cell_k=None, cell_m=None, h=1.0):
    """Assemble sum over cells of cell_k*KE_REF (stiffness) and
    cell_m*h^2*ME_REF (mass). Either weight may be None to skip it.
    Returns (K, M) as CSR matrices (None where skipped)."""
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    out = []
    for w, ref in ((cell_k, KE_REF), (cell_m, ME_REF * h * h)):
        if w is None:
            out.append(None)
            continue
        vals = (np.asarray(w, dtype=np.float64)[:, None, None] * ref[None]).ravel()
        out.append(sp.coo_matrix((vals, (rows, cols)), shape=(n_nodes, n_nodes)).tocsr())
    return tuple(out)


class FineGrid:
    """Full fine-grid Q1 discretisation of -div(kappa grad u) on [0,1]^2 with
    homogeneous Dirichlet data (paper eq. (2.1)-(2.2))."""

    def __init__(self, kappa):
        kappa = np.asarray(kappa, dtype=np.float64)
        assert kappa.ndim == 2 and kappa.shape[0] == kappa.shape[1]
        self.n = n = kappa.shape[0]
        self.h = 1.0 / n
        self.kappa = kappa
        self.n_nodes = (n + 1) ** 2
        self.conn = cell_connectivity(n, n)
        K, M = assemble(self.conn, self.n_nodes, kappa.ravel(), np.ones(n * n), self.h)
        self.K_full, self.M_full = K, M
        iy, ix = np.divmod(np.arange(self.n_nodes), n + 1)
        self.interior = np.flatnonzero((ix > 0) & (ix < n) & (iy > 0) & (iy < n))
        # full node id -> interior unknown id (-1 on the boundary)
        self.node2dof = -np.ones(self.n_nodes, dtype=np.int64)
        self.node2dof[self.interior] = np.arange(self.interior.size)
        self.A = K[self.interior][:, self.interior].tocsr()
        self.M = M[self.interior][:, self.interior].tocsr()
        self.x_nodes = ix * self.h
        self.y_nodes = iy * self.h

    @property
    def n_dof(self):
        return self.interior.size

    def load_smooth(self, fun):
        """Load vector of a smooth source: M_full @ (nodal interpolant),
        restricted to interior rows."""
        vals = fun(self.x_nodes, self.y_nodes)
        return (self.M_full @ vals)[self.interior]

    def load_cells(self, cell_mask):
        """Exact load of the indicator of a union of cells: each cell adds
        h^2/4 to each of its four corner nodes."""
        cm = np.asarray(cell_mask, dtype=np.float64).ravel()
        b = np.zeros(self.n_nodes)
        np.add.at(b, self.conn.ravel(), np.repeat(cm, 4) * (self.h * self.h / 4.0))
        return b[self.interior]

    def nodal(self, fun):
        """Nodal interpolant of fun at the interior unknowns."""
        return fun(self.x_nodes, self.y_nodes)[self.interior]
