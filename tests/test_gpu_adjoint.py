"""GPU parity of the transposed parareal (pe_adjoint, pe_tracking and the
autograd functions of the binding) against the oracle's discrete adjoint on
the same seeded inputs. Bars: FP64 path 1e-10 relative, mixed path 1e-6
relative (Euclidean on (dL/dx0, dL/dH) and on the adjoint states)."""
import numpy as np
import pytest
import torch

import oracle.adjoint as ADJ
import oracle.scheme as S
from problem import build_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-6

# ragged sizes: d1 = 18, d2 = 27
RAGGED = dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
              seed=31, source="sine_exp", u0="sine2", N=5, P=7, T=None, B=1)
# per-element interval amplitudes, R = 25 modes (the dense per-interval source table), 2 samples
ELEM = dict(n=50, n_c=5, layers=2, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
            seed=21, source="elem_interval", u0="zero", N=6, P=5, T=None, B=2, src_seed=21)
CFGS = {"ragged": RAGGED, "elem": ELEM}


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _prob(name):
    return build_problem(CFGS.get(name, name))


def _rel(a, b):
    a = np.concatenate([np.ravel(x) for x in a])
    b = np.concatenate([np.ravel(x) for x in b])
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _inputs(p, seed, track):
    """Random boundary cotangents and, for the tracking term, a trajectory y
    of the scheme (random start, random amplitudes) with its fine levels."""
    rng = np.random.default_rng(seed)
    bl = S.Blocks.from_problem(p)
    B = p["H"].shape[0]
    Xbar = rng.standard_normal((B, bl.N + 1, bl.D))
    if not track:
        return bl, Xbar, None, None, None
    dH = rng.standard_normal(p["H"].shape)
    y0 = 1e-2 * rng.standard_normal((B, bl.D))
    Yf = np.stack([ADJ.fine_trajectory(bl, S.Source(p["G"], dH[b][None], p["time_mode"], bl.N, bl.P), y0[b])
                   for b in range(B)])
    return bl, Xbar, dH, Yf, Yf[:, ::bl.P]


def _oracle(p, bl, Xbar, beta=0.0, dH=None, Yf=None):
    B = Xbar.shape[0]
    out = []
    for b in range(B):
        src = S.Source(p["G"], p["H"][b][None], p["time_mode"], bl.N, bl.P)
        Xf = ADJ.tracking_cotangents(bl, Yf[b], beta) if beta > 0 else None
        out.append(ADJ.adjoint(bl, src, Xbar[b], 0, Xbar_fine=Xf))
    x0b = np.stack([o[0] for o in out])
    Hb = np.stack([o[1] for o in out])
    lam = np.stack([o[2] for o in out])
    return x0b, Hb, lam


def _gpu(pe, p, prec, Xbar, beta=0.0, Ybnd=None, dH=None, tol=0.0, k_max=None):
    pr = pe.problem_from(p, prec)
    r = pr.adjoint(Xbar=Xbar, beta=beta, Ybnd=Ybnd, dH=dH, tol=tol, k_max=k_max, lam=True)
    pr.close()
    return r


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
@pytest.mark.parametrize("name", ["t1", "t2", "elem", "ragged"])
def test_adjoint_boundary_cotangents(name, prec, bar):
    """k_max = N: the exact transpose of the sequential fine solution."""
    pe = _pe()
    p = _prob(name)
    bl, Xbar, _, _, _ = _inputs(p, 3, False)
    x0b, Hb, lam = _oracle(p, bl, Xbar)
    r = _gpu(pe, p, prec, Xbar)
    e = _rel([r["x0bar"].cpu().numpy(), r["Hbar"].cpu().numpy()], [x0b, Hb])
    el = _rel([r["lam"].cpu().numpy()], [lam])
    print(f"{name} {prec}: grad rel err {e:.3e}, lambda rel err {el:.3e}")
    assert e <= bar and el <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
@pytest.mark.parametrize("name", ["t1", "t2", "elem"])
def test_adjoint_fine_tracking(name, prec, bar):
    """Boundary cotangents plus the fine-step tracking term, fine levels
    recomputed on the GPU from the boundary states."""
    pe = _pe()
    p = _prob(name)
    beta = 0.7
    bl, Xbar, dH, Yf, Ybnd = _inputs(p, 5, True)
    x0b, Hb, lam = _oracle(p, bl, Xbar, beta, dH, Yf)
    r = _gpu(pe, p, prec, Xbar, beta=beta, Ybnd=Ybnd, dH=dH)
    e = _rel([r["x0bar"].cpu().numpy(), r["Hbar"].cpu().numpy()], [x0b, Hb])
    el = _rel([r["lam"].cpu().numpy()], [lam])
    print(f"{name} {prec} tracking: grad rel err {e:.3e}, lambda rel err {el:.3e}")
    assert e <= bar and el <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("mixed", TOLMIX)])
@pytest.mark.parametrize("name", ["t1", "elem"])
def test_tracking_value(name, prec, bar):
    pe = _pe()
    p = _prob(name)
    beta = 1.3
    bl, _, dH, Yf, Ybnd = _inputs(p, 7, True)
    ref = np.array([0.5 * beta * bl.dt_fine * np.einsum("md,de,me->", y[1:], bl.M, y[1:]) for y in Yf])
    pr = pe.problem_from(p, prec)
    J = pr.tracking(Ybnd, dH, beta)
    pr.close()
    np.testing.assert_allclose(J, ref, rtol=bar)


def test_adjoint_coarse_only():
    """k_max = 0: the initial backward coarse sweep lam_n = Xbar_n + Phi_G^T lam_{n+1},
    Phi_G the coarse step without source formed column by column."""
    pe = _pe()
    p = _prob("t2")
    bl, Xbar, _, _, _ = _inputs(p, 9, False)
    zero = S.Source(None, None, S.TIME_FINE, bl.N, bl.P)
    Phi = np.stack([S.coarse_propagator(bl, zero, e, 0) for e in np.eye(bl.D)], axis=1)
    lam = np.zeros_like(Xbar)
    lam[:, -1] = Xbar[:, -1]
    for n in reversed(range(bl.N)):
        lam[:, n] = Xbar[:, n] + lam[:, n + 1] @ Phi
    r = _gpu(pe, p, "fp64", Xbar, k_max=0)
    assert _rel([r["lam"].cpu().numpy()], [lam]) <= 1e-12
    assert _rel([r["x0bar"].cpu().numpy()], [lam[:, 0]]) <= 1e-12


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-8), ("mixed", TOLMIX)])
def test_adjoint_stops_at_tolerance(prec, bar):
    pe = _pe()
    p = _prob("t2")
    bl, Xbar, dH, Yf, Ybnd = _inputs(p, 11, True)
    x0b, Hb, _ = _oracle(p, bl, Xbar, 1.0, dH, Yf)
    r = _gpu(pe, p, prec, Xbar, beta=1.0, Ybnd=Ybnd, dH=dH, tol=1e-11)
    e = _rel([r["x0bar"].cpu().numpy(), r["Hbar"].cpu().numpy()], [x0b, Hb])
    print(f"{prec}: iterations {r['iters']}, grad rel err {e:.3e}")
    assert r["status"] == 0
    assert np.all(r["iters"] < bl.N)
    assert e <= bar


def test_adjoint_graph_replays_are_bitwise_equal():
    """Later calls replay captured sweeps; the results do not change."""
    pe = _pe()
    p = _prob("t2")
    bl, Xbar, dH, Yf, Ybnd = _inputs(p, 13, True)
    pr = pe.problem_from(p, "mixed")
    outs = [pr.adjoint(Xbar=Xbar, beta=1.0, Ybnd=Ybnd, dH=dH, lam=True) for _ in range(3)]
    pr.close()
    for o in outs[1:]:
        assert torch.equal(o["x0bar"], outs[0]["x0bar"])
        assert torch.equal(o["Hbar"], outs[0]["Hbar"])
        assert torch.equal(o["lam"], outs[0]["lam"])


def test_adjoint_errors():
    pe = _pe()
    p = _prob("t1")
    pr = pe.problem_from(p, "fp64")
    Xbar = np.zeros((1, pr.N + 1, pr.D))
    with pytest.raises(pe.PeError, match="Ybnd"):
        pr.adjoint(Xbar=Xbar, beta=1.0)
    with pytest.raises(pe.PeError, match="k_max"):
        pr.adjoint(Xbar=Xbar, k_max=pr.N + 1)
    with pytest.raises(pe.PeError, match="beta"):
        pr.adjoint(Xbar=Xbar, beta=-1.0, Ybnd=Xbar)
    with pytest.raises(pe.PeError, match="source"):
        pr.adjoint(Xbar=np.zeros((2, pr.N + 1, pr.D)))
    pr.close()


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_autograd_parasolve(prec, bar):
    """Gradients of sum(W * X) through ParaSolve equal the oracle adjoint
    with Xbar = W."""
    pe = _pe()
    p = _prob("t2")
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(17)
    W = rng.standard_normal((p["H"].shape[0], bl.N + 1, bl.D))
    pr = pe.Problem({k: p[k] for k in ("M11", "M12", "M22", "A11", "A12", "A22")}, p["dt"], p["dt_fine"],
                    p["N"], precision=prec)
    H = torch.tensor(p["H"], dtype=torch.float64, device="cuda", requires_grad=True)
    x0 = torch.tensor(p["x0"], dtype=torch.float64, device="cuda", requires_grad=True)
    X = pe.ParaSolve.apply(H, x0, pr, p["G"], int(p["time_mode"]), 1e-13, 0.0)
    (X * torch.tensor(W, device="cuda")).sum().backward()
    x0b, Hb, _ = _oracle(p, bl, W)
    e = _rel([x0.grad.cpu().numpy(), H.grad.cpu().numpy()], [x0b, Hb])
    print(f"{prec}: autograd grad rel err {e:.3e}")
    pr.close()
    assert e <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_autograd_tracked_solve(prec, bar):
    """Terminal plus fine-step tracking loss through TrackedSolve: value and
    gradients against the oracle (reference trajectory from (H_ref, 0))."""
    pe = _pe()
    p = _prob("elem")
    bl = S.Blocks.from_problem(p)
    B = p["H"].shape[0]
    rng = np.random.default_rng(19)
    H_ref = rng.standard_normal(p["H"].shape)
    Hv = H_ref + 0.1 * rng.standard_normal(H_ref.shape)
    x0v = 0.1 * rng.standard_normal((B, bl.D)) / np.sqrt(bl.D)
    beta = 1.0
    srcs = lambda H: [S.Source(p["G"], H[b][None], p["time_mode"], bl.N, bl.P) for b in range(B)]
    Rf = np.stack([ADJ.fine_trajectory(bl, s, np.zeros(bl.D)) for s in srcs(H_ref)])
    Xf = np.stack([ADJ.fine_trajectory(bl, s, x0v[b]) for b, s in enumerate(srcs(Hv))])
    Yf = Xf - Rf
    Mt = torch.tensor(bl.M, device="cuda")

    pr = pe.Problem({k: p[k] for k in ("M11", "M12", "M22", "A11", "A12", "A22")}, p["dt"], p["dt_fine"],
                    p["N"], precision=prec)
    X_ref = torch.tensor(Rf[:, ::bl.P], device="cuda")
    H = torch.tensor(Hv, device="cuda", requires_grad=True)
    x0 = torch.tensor(x0v, device="cuda", requires_grad=True)
    X, J = pe.TrackedSolve.apply(H, x0, pr, p["G"], int(p["time_mode"]), torch.tensor(H_ref, device="cuda"),
                                 X_ref, beta, 1e-13, 0.0)
    eN = X[:, -1] - X_ref[:, -1]
    loss = 0.5 * torch.einsum("bd,de,be->", eN, Mt, eN) + J.sum()
    loss.backward()
    # oracle: terminal cotangent M e_N, tracking cotangents beta dt M y_m
    Xbar = np.zeros((B, bl.N + 1, bl.D))
    Xbar[:, -1] = Yf[:, -1] @ bl.M
    x0b, Hb, _ = _oracle(dict(p, H=Hv), bl, Xbar, beta, None, Yf)
    Jref = np.array([0.5 * beta * bl.dt_fine * np.einsum("md,de,me->", y[1:], bl.M, y[1:]) for y in Yf])
    e = _rel([x0.grad.cpu().numpy(), H.grad.cpu().numpy()], [x0b, Hb])
    print(f"{prec}: tracked autograd grad rel err {e:.3e}, J {J.detach().cpu().numpy()} vs {Jref}")
    pr.close()
    np.testing.assert_allclose(J.detach().cpu().numpy(), Jref, rtol=max(bar, 1e-12))
    assert e <= bar


_C3 = {}
_C3IN = {}


def _c3_inputs():
    """The full-size adjoint workload's problem and evaluation point."""
    if not _C3IN:
        p = build_problem("c3")
        bl = S.Blocks.from_problem(p)
        rng = np.random.default_rng(3)
        theta_ref = p["H"][0]
        theta = theta_ref + 0.1 * rng.standard_normal(theta_ref.shape)
        x0 = 0.1 * rng.standard_normal(bl.D) / np.sqrt(bl.D)
        _C3IN.update(p=p, bl=bl, theta=theta, theta_ref=theta_ref, x0=x0)
    return _C3IN


def _c3_oracle():
    """Oracle side of the full-size adjoint workload, computed once: the
    tracking error y = x - r is the fine solution for (x0, theta - theta_ref)
    (the scheme is linear), the loss 1/2 |y_NP|_M^2 + 1/2 sum_m dt_fine
    |y_m|_M^2 (beta = 1)."""
    if not _C3:
        c = _c3_inputs()
        p, bl, theta, theta_ref, x0 = c["p"], c["bl"], c["theta"], c["theta_ref"], c["x0"]
        Yf = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, theta - theta_ref)
        Xbar = np.zeros((bl.N + 1, bl.D))
        Xbar[-1] = bl.M @ Yf[-1]
        src = S.Source(p["G"], theta[None], p["time_mode"], bl.N, bl.P)
        x0b, Hb, _ = ADJ.adjoint(bl, src, Xbar, Xbar_fine=ADJ.tracking_cotangents(bl, Yf, 1.0))
        J = 0.5 * bl.dt_fine * np.einsum("md,de,me->", Yf[1:], bl.M, Yf[1:])
        _C3.update(p=p, bl=bl, theta=theta, theta_ref=theta_ref, x0=x0, Yf=Yf, x0b=x0b, Hb=Hb, J=J)
    return _C3


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_full_size_adjoint_c3(prec, bar):
    """Full-size adjoint workload (d1 = 800, d2 = 1200, N = 64 x P = 64,
    400 x 64 per-element interval amplitudes): forward parareal for y and
    transposed parareal on the GPU, against the oracle's adjoint of the
    sequential fine solution."""
    pe = _pe()
    c = _c3_oracle()
    p, bl = c["p"], c["bl"]
    pr = pe.problem_from(dict(p, H=(c["theta"] - c["theta_ref"])[None]), prec)
    tol = 1e-13 if prec == "fp64" else 1e-9
    Y, it_f, _, st = pr.solve(c["x0"][None], tol=tol, norm="rel")
    assert st == 0
    Mt = torch.tensor(bl.M, device="cuda")
    Xbar = torch.zeros_like(Y)
    Xbar[:, -1] = Y[:, -1] @ Mt
    dH = torch.tensor((c["theta"] - c["theta_ref"])[None], device="cuda")
    r = pr.adjoint(Xbar=Xbar, beta=1.0, Ybnd=Y, dH=dH, tol=tol)
    J = pr.tracking(Y, dH, 1.0)
    pr.close()
    e = _rel([r["x0bar"].cpu().numpy()[0], r["Hbar"].cpu().numpy()[0]], [c["x0b"], c["Hb"]])
    ey = _rel([Y.cpu().numpy()[0]], [c["Yf"][::bl.P]])
    print(f"c3 {prec}: forward iterations {it_f}, adjoint iterations {r['iters']}, y rel err {ey:.3e}, "
          f"grad rel err {e:.3e}, J {J[0]:.6e} vs {c['J']:.6e}")
    assert r["status"] == 0
    assert e <= bar
    np.testing.assert_allclose(J[0], c["J"], rtol=max(bar, 1e-12))


@pytest.mark.parametrize("prec,bar", [("fp64", TOL64), ("mixed", TOLMIX)])
def test_adjoint_full_space_no_explicit_part(prec, bar):
    """d2 = 0 (V_H1 = the whole fine Q1 space): the transposed scheme is
    transposed backward Euler; boundary cotangents plus fine-step tracking."""
    pe = _pe()
    from problem.fem import FineGrid
    n, P, N = 12, 5, 4
    rng = np.random.default_rng(23)
    fine = FineGrid(np.exp(2 * rng.standard_normal((n, n))))
    M, A = fine.M.toarray(), fine.A.toarray()
    d1 = M.shape[0]
    dt = 1e-2
    z = np.zeros((d1, 0))
    bl = S.Blocks(M, z, np.zeros((0, 0)), A, z, np.zeros((0, 0)), dt, dt / P, N)
    G = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * y)[:, None]
    H = rng.standard_normal((1, 1, N))
    Xbar = rng.standard_normal((1, N + 1, d1))
    dH = rng.standard_normal((1, 1, N))
    Yf = ADJ.fine_trajectory(bl, S.Source(G, dH, S.TIME_INTERVAL, N, P), 0.1 * rng.standard_normal(d1))
    src = S.Source(G, H, S.TIME_INTERVAL, N, P)
    x0b, Hb, lam = ADJ.adjoint(bl, src, Xbar[0], Xbar_fine=ADJ.tracking_cotangents(bl, Yf, 1.0))
    pr = pe.Problem(dict(M11=M, M12=z, M22=np.zeros((0, 0)), A11=A, A12=z, A22=np.zeros((0, 0))),
                    dt, dt / P, N, prec)
    pr.set_source(G, H, "interval")
    r = pr.adjoint(Xbar=Xbar, beta=1.0, Ybnd=Yf[::P][None], dH=dH, lam=True)
    pr.close()
    e = _rel([r["x0bar"].cpu().numpy()[0], r["Hbar"].cpu().numpy()[0]], [x0b, Hb])
    el = _rel([r["lam"].cpu().numpy()[0]], [lam])
    print(f"d2 = 0 {prec}: grad rel err {e:.3e}, lambda rel err {el:.3e}")
    assert e <= bar and el <= bar


def test_full_size_adjoint_finite_differences_fp64():
    """The GPU gradient of the full-size adjoint workload's loss against
    central differences (h = 1e-6) of that loss evaluated by GPU forward
    solves (k = N: the sequential fine solution) and pe_tracking, along 8
    random unit directions and 16 random coordinates of (x0, theta); the
    loss is quadratic, so only rounding separates the two."""
    pe = _pe()
    c = _c3_inputs()
    p, bl = c["p"], c["bl"]
    dth0 = c["theta"] - c["theta_ref"]
    Mt = torch.tensor(bl.M, device="cuda")
    pr = pe.problem_from(dict(p, H=dth0[None]), "fp64")

    def loss(dx0, dth):
        pr.set_source(p["G"], (dth0 + dth)[None], "interval")
        Y, _, _, _ = pr.solve((c["x0"] + dx0)[None], tol=0.0)
        J = pr.tracking(Y, torch.tensor((dth0 + dth)[None], device="cuda"), 1.0)[0]
        yN = Y[0, -1]
        return 0.5 * float(yN @ (Mt @ yN)) + J, Y

    L0, Y = loss(np.zeros(bl.D), np.zeros(dth0.shape))
    Xbar = torch.zeros_like(Y)
    Xbar[:, -1] = Y[:, -1] @ Mt
    r = pr.adjoint(Xbar=Xbar, beta=1.0, Ybnd=Y, dH=torch.tensor(dth0[None], device="cuda"))
    gx, gh = r["x0bar"].cpu().numpy()[0], r["Hbar"].cpu().numpy()[0]
    rng = np.random.default_rng(31)
    dirs = []
    for _ in range(8):
        dx, dH = rng.standard_normal(bl.D), rng.standard_normal(dth0.shape)
        nrm = np.sqrt(np.sum(dx ** 2) + np.sum(dH ** 2))
        dirs.append((dx / nrm, dH / nrm))
    for idx in rng.choice(bl.D + dth0.size, size=16, replace=False):
        dx, dH = np.zeros(bl.D), np.zeros(dth0.shape)
        if idx < bl.D:
            dx[idx] = 1.0
        else:
            dH.flat[idx - bl.D] = 1.0
        dirs.append((dx, dH))
    h = 1e-6
    fd, ad = [], []
    for dx, dH in dirs:
        lp, _ = loss(h * dx, h * dH)
        lm, _ = loss(-h * dx, -h * dH)
        fd.append((lp - lm) / (2 * h))
        ad.append(float(np.sum(dx * gx) + np.sum(dH * gh)))
    pr.close()
    fd, ad = np.array(fd), np.array(ad)
    print("FD vs adjoint, max rel diff %.3e (L = %.3e)" % (np.max(np.abs(fd - ad) / np.abs(ad).max()), L0))
    np.testing.assert_allclose(fd, ad, rtol=1e-5, atol=1e-5 * np.abs(ad).max())
