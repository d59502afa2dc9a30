"""Graph replays of the sweeps against eager launches: bitwise equal results
on several replays with other eager work and synchronisations in between
(tile configurations fixed by the heuristic: PE_AUTOTUNE=0)."""
import os

import numpy as np
import pytest
import torch

import oracle.scheme as S
from problem import build_problem

pytestmark = pytest.mark.gpu


def _make(p, prec, graphs):
    import paper_2411_09244_amd as pe
    old = {k: os.environ.get(k) for k in ("PE_GRAPHS", "PE_AUTOTUNE")}
    os.environ["PE_GRAPHS"] = "1" if graphs else "0"
    os.environ["PE_AUTOTUNE"] = "0"
    try:
        return pe.problem_from(p, prec)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("name", ["c0", "t2"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager(name, prec):
    p = build_problem(name)
    eager = _make(p, prec, graphs=False)
    graph = _make(p, prec, graphs=True)
    ref = eager.solve(p["x0"], tol=1e-7, norm="rel")
    Xref = ref[0].clone()
    other = build_problem("t1")
    side = _make(other, "fp64", graphs=False)
    for rep in range(4):
        X, iters, hist, st = graph.solve(p["x0"], tol=1e-7, norm="rel")
        assert np.array_equal(iters, ref[1]), rep
        assert torch.equal(X, Xref), (rep, (X - Xref).abs().max().item())
        # eager work and synchronisation between replays
        side.solve(other["x0"], tol=0.0, k_max=2)
        torch.cuda.synchronize()
    bl = S.Blocks.from_problem(p)
    assert all(np.isfinite(X.cpu().numpy()).ravel())
    eager.close(), graph.close(), side.close()
