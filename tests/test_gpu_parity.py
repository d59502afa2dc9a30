"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs. Bars: FP64 path 1e-10 relative (M-norm), mixed path 1e-6
relative; the coarse propagator and norms are FP64 in both paths (1e-12)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle.scheme as S
from problem import build_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-6

# ragged sizes: d1 = 18, d2 = 27 (not multiples of the 8/64 paddings)
RAGGED = dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
              seed=31, source="sine_exp", u0="sine2", N=5, P=7, T=None, B=1)


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _prob(name):
    return build_problem(RAGGED if name == "ragged" else name)


def _colwise_rel(bl, Y, Yref):
    """max over columns of |Y - Yref|_M / max_c |Yref_c|_M."""
    scale = max(S.m_norm(bl, y) for y in Yref) or 1.0
    return max(S.m_norm(bl, a - b) for a, b in zip(Y, Yref)) / scale


def _random_states(prob, seed, B, N):
    rng = np.random.default_rng(seed)
    D = prob["d1"] + prob["d2"]
    x = rng.standard_normal((B, N, D))
    # scale like the solution: the state size of the sequential solution
    return x * 1e-3


@pytest.mark.parametrize("name", ["t0", "t1", "ragged"])
def test_mass_norms(name):
    pe = _pe()
    p = _prob(name)
    bl = S.Blocks.from_problem(p)
    pr = pe.problem_from(p, "fp64")
    X = np.random.default_rng(1).standard_normal((7, bl.D))
    got = pr.mass_norms(X)
    ref = np.array([S.m_norm(bl, x) for x in X])
    np.testing.assert_allclose(got, ref, rtol=1e-13)


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged"])
def test_coarse_propagator(name):
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    B, N = p["B"], p["N"]
    Xin = _random_states(p, 2, B, N)
    for prec in ("fp64", "mixed"):
        pr = pe.problem_from(p, prec)
        Y = pr.coarse(Xin).cpu().numpy()
        for b in range(B):
            ref = np.stack([S.coarse_propagator(bl, src, Xin[b, n], n, b) for n in range(N)])
            assert _colwise_rel(bl, Y[b], ref) < 1e-12, (name, prec, b)


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged", "t1n", "t1p"])
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_fine_propagator(name, prec, tol):
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    B, N = p["B"], p["N"]
    Xin = _random_states(p, 3, B, N)
    pr = pe.problem_from(p, prec)
    Y = pr.fine(Xin).cpu().numpy()
    for b in range(B):
        ref = S.fine_propagator_cols(bl, src, Xin[b].T.copy(), list(range(N)), [b] * N).T
        err = _colwise_rel(bl, Y[b], ref)
        assert err < tol, (name, prec, b, err)


def _oracle_parareal(p, k_max, tol=0.0, rel=False):
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    return bl, [S.parareal(bl, src, p["x0"][b], tol, k_max=k_max, b=b, rel=rel) for b in range(p["B"])]


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged", "t1n", "t1p"])
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_solve_equal_iteration(name, prec, tol):
    """GPU iterate k vs oracle iterate k (fixed k, no early stop)."""
    pe = _pe()
    p = _prob(name)
    k = min(3, p["N"])
    bl, refs = _oracle_parareal(p, k)
    pr = pe.problem_from(p, prec)
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=k)
    X = X.cpu().numpy()
    assert (iters == k).all()
    for b, r in enumerate(refs):
        err = S.rel_l2_M(bl, X[b], r["X"][k])
        assert err < tol, (name, prec, b, err)
        # a jump is a difference of two states: its error is bounded by the
        # state error, so it is measured against the state scale
        scale = max(S.m_norm(bl, x) for x in r["X"][k])
        assert np.abs(hist[b] - r["J"]).max() <= tol * scale, (hist[b], r["J"])


@pytest.mark.parametrize("name", ["t1", "c0", "t1n"])
def test_solve_exact_after_n_iterations(name):
    """k = N reproduces the sequential fine solution (finite termination)."""
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    Xs = S.fine_composition(bl, src, p["x0"][0])
    pr = pe.problem_from(p, "fp64")
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=p["N"])
    assert S.rel_l2_M(bl, X[0].cpu().numpy(), Xs) < TOL64


@pytest.mark.parametrize("name", ["t1", "c0", "t2"])
def test_stopping_test_iterations_match_oracle(name):
    pe = _pe()
    p = _prob(name)
    bl, refs = _oracle_parareal(p, None, tol=1e-7, rel=True)
    for prec in ("fp64", "mixed"):
        pr = pe.problem_from(p, prec)
        X, iters, hist, st = pr.solve(p["x0"], tol=1e-7, norm="rel")
        assert st == 0
        for b, r in enumerate(refs):
            assert iters[b] == r["K"], (prec, b, iters[b], r["K"], hist[b])
            err = S.rel_l2_M(bl, X[b].cpu().numpy(), r["X"][r["K"]])
            assert err < (TOL64 if prec == "fp64" else TOLMIX), (prec, b, err)


def test_full_space_no_explicit_part():
    """d2 = 0 (V_H1 = whole fine Q1 space): the path is fine backward Euler."""
    pe = _pe()
    from problem.fem import FineGrid
    n, P, N = 12, 5, 3
    rng = np.random.default_rng(7)
    fine = FineGrid(np.exp(2 * rng.standard_normal((n, n))))
    M, A = fine.M.toarray(), fine.A.toarray()
    d1 = M.shape[0]
    dt = 1e-2
    z = np.zeros((d1, 0))
    bl = S.Blocks(M, z, np.zeros((0, 0)), A, z, np.zeros((0, 0)), dt, dt / P, N)
    G = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * y)[:, None]
    H = rng.standard_normal((1, 1, N))
    src = S.Source(G, H, S.TIME_INTERVAL, N, P)
    x0 = rng.standard_normal(d1) * 0.1
    Xs = S.fine_composition(bl, src, x0)
    pr = pe.Problem(dict(M11=M, M12=z, M22=np.zeros((0, 0)), A11=A, A12=z, A22=np.zeros((0, 0))),
                    dt, dt / P, N, "fp64")
    pr.set_source(G, H, "interval")
    X, iters, hist, st = pr.solve(x0[None], tol=0.0, k_max=N)
    assert S.rel_l2_M(bl, X[0].cpu().numpy(), Xs) < TOL64


def test_bitwise_deterministic():
    pe = _pe()
    p = _prob("c0")
    for prec in ("fp64", "mixed"):
        pr = pe.problem_from(p, prec)
        X1 = pr.solve(p["x0"], tol=0.0, k_max=3)[0].clone()
        X2 = pr.solve(p["x0"], tol=0.0, k_max=3)[0]
        assert torch.equal(X1, X2), prec


def test_error_paths():
    pe = _pe()
    from paper_2411_09244_amd import _lib
    p = _prob("t0")
    blocks = {k: p[k].copy() for k in ("M11", "M12", "M22", "A11", "A12", "A22")}
    # not SPD: flip the sign of M11 (K = M11/dt + A11 loses definiteness)
    bad = dict(blocks, M11=-blocks["M11"] * 1e6)
    with pytest.raises(pe.PeError) as ei:
        pe.Problem(bad, p["dt"], p["dt_fine"], p["N"])
    assert ei.value.status == _lib.PE_ERR_NOT_SPD
    # asymmetric A11
    asym = dict(blocks)
    asym["A11"] = blocks["A11"].copy()
    asym["A11"][0, 1] += 1e-3 * np.abs(blocks["A11"]).max()
    with pytest.raises(pe.PeError) as ei:
        pe.Problem(asym, p["dt"], p["dt_fine"], p["N"])
    assert ei.value.status == _lib.PE_ERR_ARG
    # non-integer step ratio
    with pytest.raises(pe.PeError) as ei:
        pe.Problem(blocks, p["dt"], p["dt"] / 3.5, p["N"])
    assert ei.value.status == _lib.PE_ERR_ARG
    # NaN in the initial state
    pr = pe.problem_from(p, "fp64")
    x0 = p["x0"].copy()
    x0[0, 3] = np.nan
    with pytest.raises(pe.PeError) as ei:
        pr.solve(x0, tol=1e-12, k_max=2)
    assert ei.value.status == _lib.PE_ERR_NONFINITE
    # k_max > N
    with pytest.raises(pe.PeError):
        pr.solve(p["x0"], tol=0.0, k_max=p["N"] + 1)
    # unreachable tolerance -> warning, last iterate returned
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=2)
    assert st == _lib.PE_WARN_NOT_CONVERGED and iters[0] == 2


@pytest.fixture(scope="module")
def c1_reference():
    """The 200x200 / 20x20 workload (d1 = 800, d2 = 1200, N = 64, P = 64) and
    the oracle's sequential fine solution on all 64 intervals."""
    p = build_problem("c1")
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    return p, bl, S.fine_composition(bl, src, p["x0"][0])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_full_size_c1(c1_reference, prec, tol):
    """Converged GPU iterate (rel tol 1e-7, the benchmark's launch
    configuration) vs the oracle's sequential fine solution, every interval."""
    pe = _pe()
    p, bl, Xs = c1_reference
    pr = pe.problem_from(p, prec)
    X, iters, hist, st = pr.solve(p["x0"], tol=1e-7, norm="rel")
    assert st == 0 and 1 <= iters[0] <= p["N"]
    X = X[0].cpu().numpy()
    err = S.rel_l2_M(bl, X, Xs)
    print(f"c1 {prec}: iterations {iters[0]}, rel L2 vs sequential fine solution {err:.3e}, "
          f"jumps {hist[0][:iters[0]]}")
    assert err < tol


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_persistent_fine_sweep(prec, bar, monkeypatch):
    """The opt-in persistent fine sweep (one cooperative launch per sweep,
    grid barriers between the steps) against the oracle: the fine propagator
    and a full solve, including the full-size 64-column workload."""
    pe = _pe()
    monkeypatch.setenv("PE_PERSISTENT", "1")
    for name in ("t1", "c1"):
        p = _prob(name)
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        pr = pe.problem_from(p, prec)
        X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=2)
        prof = None
        pr.profile(True)
        Y = pr.fine(X[:, :-1].contiguous())
        prof = pr.profile_read()
        pr.close()
        assert prof["fine_sweep"][1] == 1 and prof["fine_step"][1] == 0, prof
        ref = S.fine_propagator_cols(bl, src, X[0, :-1].cpu().numpy().T, list(range(bl.N)), [0] * bl.N).T
        e = _colwise_rel(bl, Y[0].cpu().numpy(), ref)
        print(f"{name} {prec}: persistent F vs oracle {e:.3e}")
        assert e <= bar


def test_probe_peaks_sane():
    # measured matrix-core and HBM peaks: positive and not above the
    # datasheet values (157.3 / 78.6 TFLOP/s, 8 TB/s) by more than 10 %
    pe = _pe()
    pk = pe.probe_peaks()
    print(pk)
    assert 0 < pk["fp32_mfma_tflops"] < 1.1 * 157.3
    assert 0 < pk["fp64_mfma_tflops"] < 1.1 * 78.6
    assert 0 < pk["hbm_copy_tbps"] < 1.1 * 8.0


WSK_CFGS = ["32,4,1", "32,8,2", "16,4,4", "16,8,1"]


@pytest.mark.parametrize("cfg", WSK_CFGS)
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_wave_split_k_kernel(cfg, prec, tol, monkeypatch):
    """Every product whose state columns fit one 64-row tile forced onto the
    wave-split-K kernel (cfg = operator rows per tile, waves per work-group,
    K splits): the fine propagator against the oracle on ragged and tiled
    sizes (including the 200x200 workload), and parareal at equal k."""
    pe = _pe()
    monkeypatch.setenv("PE_FORCE_WSK", cfg)
    for name in ("t1", "ragged", "c0", "c1"):
        p = _prob(name)
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        B, N = p["B"], p["N"]
        print(f"[wsk] {cfg} {prec} {name}", flush=True)
        Xin = _random_states(p, 3, B, N)
        pr = pe.problem_from(p, prec)
        Y = pr.fine(Xin).cpu().numpy()
        tiles = pr.last_tiles("fine_step")
        assert tiles[2] == -int(cfg.split(",")[1]) and tiles[1] == int(cfg.split(",")[0]), tiles
        for b in range(B):
            ref = S.fine_propagator_cols(bl, src, Xin[b].T.copy(), list(range(N)), [b] * N).T
            err = _colwise_rel(bl, Y[b], ref)
            print(f"  F vs oracle b={b}: {err:.3e}")
            assert err < tol, (name, cfg, prec, b, err)
        if name in ("t1", "ragged"):
            X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=3)
            _, refs = _oracle_parareal(p, 3)
            for b in range(B):
                err = S.rel_l2_M(bl, X[b].cpu().numpy(), refs[b]["X"][3])
                print(f"  parareal k=3 vs oracle b={b}: {err:.3e}")
                assert err < tol, (name, cfg, prec, b, err)
        pr.close()


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "ragged"])
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_coarse_scan_matches_sequential(name, prec, tol, monkeypatch):
    """The one-sample coarse sweep as a doubling scan (default) against the
    sequential sweep (PE_COARSE_SCAN=0) and the oracle at equal k, with N = 6,
    8, 8, 5 intervals (3, 3, 3 and 3 scan levels; the rows before each
    shift read the zero rows in front of the buffer)."""
    pe = _pe()
    p = _prob(name)
    k = min(3, p["N"])
    bl, refs = _oracle_parareal(p, k)
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("PE_COARSE_SCAN", mode)
        pr = pe.problem_from(p, prec)
        X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=k)
        out[mode] = X.cpu().numpy()
        pr.close()
    for b, r in enumerate(refs):
        e_scan = S.rel_l2_M(bl, out["1"][b], r["X"][k])
        e_seq = S.rel_l2_M(bl, out["0"][b], r["X"][k])
        e_ab = S.rel_l2_M(bl, out["1"][b], out["0"][b])
        print(f"{name} {prec}: scan {e_scan:.3e}, sequential {e_seq:.3e}, scan vs sequential {e_ab:.3e}")
        assert e_scan < tol and e_seq < tol and e_ab < tol


TILE_CFGS = ["64,32,1,8", "32,64,0,4", "64,64,0,2", "128,64,0,3", "128,128,0,1"]


@pytest.mark.parametrize("cfg", TILE_CFGS)
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_forced_tile_configurations(cfg, prec, tol, monkeypatch):
    """Every product of more than 4 state columns forced onto one tile
    configuration (cfg = state rows, operator rows per tile, K-depth flag,
    K splits), so that ragged last tiles, tiles mostly past the state rows
    (128-row tiles over 64 or 65 state rows: matrix-core blocks wholly in the
    padding are skipped) and split-K planes are all exercised: the fine
    propagator against the oracle on ragged and tiled sizes up to the 200x200
    workload, and parareal at equal k on two of them (fine steps, anchors,
    stopping-test norms and coarse scans run through the same products)."""
    pe = _pe()
    monkeypatch.setenv("PE_FORCE_TILES", cfg)
    for name in ("t1", "ragged", "c0", "c1"):
        p = _prob(name)
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        B, N = p["B"], p["N"]
        print(f"[tiles] {cfg} {prec} {name}", flush=True)
        Xin = _random_states(p, 5, B, N)
        pr = pe.problem_from(p, prec)
        Y = pr.fine(Xin).cpu().numpy()
        tiles = pr.last_tiles("fine_step")
        want = [int(v) for v in cfg.split(",")]
        assert tiles[0] == want[0] and tiles[1] == want[1] and tiles[3] == want[3], tiles
        for b in range(B):
            ref = S.fine_propagator_cols(bl, src, Xin[b].T.copy(), list(range(N)), [b] * N).T
            err = _colwise_rel(bl, Y[b], ref)
            print(f"  F vs oracle b={b}: {err:.3e}")
            assert err < tol, (name, cfg, prec, b, err)
        if name in ("t1", "ragged"):
            X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=3)
            _, refs = _oracle_parareal(p, 3)
            for b in range(B):
                err = S.rel_l2_M(bl, X[b].cpu().numpy(), refs[b]["X"][3])
                print(f"  parareal k=3 vs oracle b={b}: {err:.3e}")
                assert err < tol, (name, cfg, prec, b, err)
        pr.close()
