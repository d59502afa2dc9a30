"""GPU parity of batches of different problems (pe_batch_*): every problem
of a ragged batch (different d1, d2, N, sources and sample counts, same
step ratio P) against the FP64 oracle, per problem and per sample. Bars:
FP64 path 1e-10, mixed path 1e-6 relative (M-norm over all boundaries)."""
import numpy as np
import pytest
import torch

import oracle.scheme as S
from problem import build_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-6

# step ratio P = 4 for all; sizes from d1 = 8 to d1 = 72
BATCH = [
    dict(n=20, n_c=2, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e4, seed=40,
         source="one", u0="zero", N=6, P=4, T=None, B=1),
    dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="channels", n_h=2, n_v=2, contrast=1e6, seed=41,
         source="sine_exp", u0="sine2", N=9, P=4, T=None, B=1),
    dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5, seed=42,
         source="sine_exp", u0="sine2", N=5, P=4, T=None, B=1),
    dict(n=60, n_c=6, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0, corr=0.05, n_h=2, n_v=2,
         contrast=1e6, incl=0.2, seed=43, source="fourier8_interval", u0="zero", N=12, P=4, T=None, B=3,
         src_seed=43),
    dict(n=50, n_c=5, layers=2, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5, seed=44,
         source="elem_interval", u0="zero", N=7, P=4, T=None, B=2, src_seed=44),
]


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _setup(pe, prec, cfgs=BATCH):
    probs = [build_problem(c) for c in cfgs]
    prs = [pe.problem_from(p, prec) for p in probs]
    return probs, prs


def _rel(bl, X, Xref):
    num = sum(S.m_norm(bl, a - b) ** 2 for a, b in zip(X, Xref))
    den = sum(S.m_norm(bl, b) ** 2 for b in Xref)
    return np.sqrt(num / den)


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_batch_exact_at_k_equal_n(prec, bar):
    """tol = 0: every problem iterates until its jump is exactly zero or k = N_i;
    each result is then its sequential fine solution."""
    pe = _pe()
    probs, prs = _setup(pe, prec)
    bt = pe.Batch(prs)
    Xs, its, st = bt.solve([p["x0"] for p in probs], tol=0.0)
    for p, X, it in zip(probs, Xs, its):
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        for b in range(X.shape[0]):
            ref = S.fine_composition(bl, src, p["x0"][b], b)
            e = _rel(bl, X[b].cpu().numpy(), ref)
            print(f"{prec} d1={p['d1']} N={p['N']} sample {b}: iterations {it[b]}, rel err {e:.3e}")
            assert 1 <= it[b] <= p["N"]
            assert e <= bar
    bt.close()


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", TOLMIX)])
def test_batch_stopping_test_per_problem(prec, bar):
    """Relative stopping test per sample: the iterate equals the oracle's
    parareal iterate at the same k, and k is the oracle's k."""
    pe = _pe()
    probs, prs = _setup(pe, prec)
    bt = pe.Batch(prs)
    tol = 1e-8
    Xs, its, st = bt.solve([p["x0"] for p in probs], tol=tol, norm="rel")
    assert st == 0
    for p, X, it in zip(probs, Xs, its):
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        for b in range(X.shape[0]):
            r = S.parareal(bl, src, p["x0"][b], tol, b=b, rel=True)
            e = _rel(bl, X[b].cpu().numpy(), r["X"][it[b]])
            print(f"{prec} d1={p['d1']} N={p['N']} sample {b}: iterations {it[b]} (oracle {r['K']}), "
                  f"rel err vs oracle iterate {e:.3e}")
            assert abs(int(it[b]) - r["K"]) <= (0 if prec == "fp64" else 1)
            assert e <= bar
    bt.close()


def test_batch_matches_single_problem_solves():
    """The batch and one pe_solve per problem agree to rounding."""
    pe = _pe()
    probs, prs = _setup(pe, "fp64")
    bt = pe.Batch(prs)
    Xs, its, _ = bt.solve([p["x0"] for p in probs], tol=1e-9, norm="rel")
    for p, pr, X, it in zip(probs, prs, Xs, its):
        Y, it1, _, _ = pr.solve(p["x0"], tol=1e-9, norm="rel")
        np.testing.assert_array_equal(it, it1)
        bl = S.Blocks.from_problem(p)
        for b in range(X.shape[0]):
            assert _rel(bl, X[b].cpu().numpy(), Y[b].cpu().numpy()) <= 1e-12
    bt.close()


def test_batch_replays_are_bitwise_equal():
    pe = _pe()
    probs, prs = _setup(pe, "mixed")
    bt = pe.Batch(prs)
    outs = [bt.solve([p["x0"] for p in probs], tol=1e-8, norm="rel") for _ in range(3)]
    for Xs, its, _ in outs[1:]:
        for a, b in zip(Xs, outs[0][0]):
            assert torch.equal(a, b)
        for a, b in zip(its, outs[0][1]):
            np.testing.assert_array_equal(a, b)
    bt.close()


def test_batch_k_max_caps_each_problem():
    pe = _pe()
    probs, prs = _setup(pe, "fp64")
    bt = pe.Batch(prs)
    Xs, its, st = bt.solve([p["x0"] for p in probs], tol=0.0, k_max=3)
    assert st == 1  # not converged
    for p, X, it in zip(probs, Xs, its):
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        r = S.parareal(bl, src, p["x0"][0], 0.0, k_max=3, b=0)
        assert it[0] == 3
        assert _rel(bl, X[0].cpu().numpy(), r["X"][3]) <= TOL64
    bt.close()


def test_batch_errors():
    pe = _pe()
    probs = [build_problem(BATCH[0]), build_problem(dict(BATCH[1], P=8))]
    prs = [pe.problem_from(p, "fp64") for p in probs]
    with pytest.raises(pe.PeError, match="step ratio"):
        pe.Batch(prs)
    prs2 = [pe.problem_from(probs[0], "fp64"), pe.problem_from(probs[0], "mixed")]
    with pytest.raises(pe.PeError, match="precision"):
        pe.Batch(prs2)


def test_batch_with_full_space_problem():
    """A d2 = 0 problem (V_H1 = the whole fine space) inside a ragged batch."""
    pe = _pe()
    from problem.fem import FineGrid
    n, P, N = 12, 4, 5
    rng = np.random.default_rng(29)
    fine = FineGrid(np.exp(2 * rng.standard_normal((n, n))))
    M, A = fine.M.toarray(), fine.A.toarray()
    d1 = M.shape[0]
    dt = 1e-2
    z = np.zeros((d1, 0))
    bl0 = S.Blocks(M, z, np.zeros((0, 0)), A, z, np.zeros((0, 0)), dt, dt / P, N)
    G = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * y)[:, None]
    H = rng.standard_normal((1, 1, N))
    x0 = rng.standard_normal(d1) * 0.1
    for prec, bar in (("fp64", TOL64), ("mixed", TOLMIX)):
        pr0 = pe.Problem(dict(M11=M, M12=z, M22=np.zeros((0, 0)), A11=A, A12=z, A22=np.zeros((0, 0))),
                         dt, dt / P, N, prec)
        pr0.set_source(G, H, "interval")
        probs, prs = _setup(pe, prec, BATCH[:3])
        bt = pe.Batch([pr0] + prs)
        Xs, its, st = bt.solve([x0[None]] + [p["x0"] for p in probs], tol=0.0)
        ref = S.fine_composition(bl0, S.Source(G, H, S.TIME_INTERVAL, N, P), x0)
        e0 = _rel(bl0, Xs[0][0].cpu().numpy(), ref)
        print(f"{prec}: d2 = 0 member rel err {e0:.3e}, iterations {its[0]}")
        assert e0 <= bar
        for p, X in zip(probs, Xs[1:]):
            bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
            assert _rel(bl, X[0].cpu().numpy(), S.fine_composition(bl, src, p["x0"][0], 0)) <= bar
        bt.close()
