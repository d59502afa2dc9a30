"""Pins of the NLMC spaces (Section 3.2): the constraints of eq. (3.6), the
first-order optimality of the constrained energy minimisation, the fracture
count against a library connected-component labelling, the two splits
spanning one space, the dimensions of the printed split, and the contrast
dependence of the stability quantities (lambda2, gamma, the stable step)."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse as sp

from problem import build, nlmc
from problem.cem import CoarseGrid
from problem.fem import FineGrid


def _setup(contrast=1e6, split="nlmc_fm"):
    cfg = dict(build.CONFIGS["t1n"])
    cfg["contrast"] = contrast
    cfg["split"] = split
    kappa = build.make_medium(cfg)
    fine = FineGrid(kappa)
    cg = CoarseGrid(fine, cfg["n_c"])
    regions = nlmc.fracture_regions(cg, np.sqrt(contrast))
    return cfg, fine, cg, regions


def test_fracture_count_matches_library_labelling():
    cfg, fine, cg, regions = _setup()
    high = (fine.kappa >= 1e3)
    for e in range(cg.n_elem):
        ey, ex = divmod(e, cg.n_c)
        block = high[ey * cg.m:(ey + 1) * cg.m, ex * cg.m:(ex + 1) * cg.m]
        _, count = ndi.label(block)      # 4-connectivity
        assert len(regions[e][1]) == count, e
        assert sum(len(f) for f in regions[e][1]) + len(regions[e][0]) == cg.m * cg.m


def test_constraints_and_optimality():
    cfg, fine, cg, regions = _setup()
    psis, res = nlmc.nlmc_basis(cg, regions, cfg["layers"], return_checks=True)
    assert max(res) < 1e-6
    # optimality on one interior patch: A psi lies in the range of C^T
    i = cg.n_elem // 2 + 1
    elems, free_ids = cg.patch(i, cfg["layers"])
    lookup = -np.ones(fine.n_nodes, dtype=np.int64)
    lookup[free_ids] = np.arange(free_ids.size)
    rows = []
    for k in elems:
        mat, fr = regions[k]
        for cells in [mat] + fr:
            c, v = nlmc._region_row(fine, cells, lookup)
            r = np.zeros(free_ids.size)
            np.add.at(r, c, v)
            rows.append(r)
    C = np.array(rows)
    A = fine.K_full.tocsr()[free_ids][:, free_ids]
    ids, psi = psis[i]
    assert np.array_equal(ids, free_ids)
    Ap = A @ psi
    mu, *_ = np.linalg.lstsq(C.T, Ap, rcond=None)
    assert np.linalg.norm(C.T @ mu - Ap) <= 1e-8 * np.linalg.norm(Ap)


def test_split_dimensions_and_common_span():
    cfg, fine, cg, regions = _setup()
    psis = nlmc.nlmc_basis(cg, regions, cfg["layers"])
    L = sum(len(r[1]) for r in regions)
    P1, P2 = nlmc.nlmc_split(cg, psis, "paper")
    F1, F2 = nlmc.nlmc_split(cg, psis, "fm")
    assert (P1.shape[1], P2.shape[1]) == (L - 1, cg.n_elem + 1)
    assert (F1.shape[1], F2.shape[1]) == (L, cg.n_elem)
    Pa = sp.hstack([P1, P2]).toarray()
    Fa = sp.hstack([F1, F2]).toarray()
    Q, _ = np.linalg.qr(Fa)
    assert np.linalg.norm(Pa - Q @ (Q.T @ Pa)) <= 1e-9 * np.linalg.norm(Pa)
    Q, _ = np.linalg.qr(Pa)
    assert np.linalg.norm(Fa - Q @ (Q.T @ Fa)) <= 1e-9 * np.linalg.norm(Fa)


def _diag(contrast, split):
    cfg, fine, cg, regions = _setup(contrast, split)
    psis = nlmc.nlmc_basis(cg, regions, cfg["layers"])
    P1, P2 = nlmc.nlmc_split(cg, psis, "paper" if split == "nlmc" else "fm")
    return build.diagnostics(build.project_blocks(fine, P1, P2), with_cond=False)


def test_fracture_matrix_split_is_contrast_independent():
    # Section 3.2: with fracture functions in V_H1 and matrix functions in
    # V_H2 the stability condition dt lambda2 <= 1 - gamma^2 does not depend
    # on the channel contrast
    d = [_diag(c, "nlmc_fm") for c in (1e2, 1e4, 1e6)]
    dts = [x["dt_max"] for x in d]
    assert max(dts) / min(dts) < 1.05
    assert all(x["gamma2"] < 0.3 for x in d)


def test_printed_split_gamma_contrast_independent():
    # the printed split (psi_bar in V_H2): gamma does not depend on the
    # contrast, but lambda2 grows with it (psi_bar carries the fracture
    # functions' gradients inside the channels)
    d = [_diag(c, "nlmc") for c in (1e2, 1e4, 1e6)]
    g = [x["gamma2"] for x in d]
    assert max(g) - min(g) < 0.01 and max(g) < 0.6
    assert d[2]["lambda2"] > 100 * d[0]["lambda2"]
