"""GPU parity of the ragged batch of different solves (the batched workload:
every solve its own medium, coarse grid 8x8..32x32, contrast, interval count
and source, spaces built on the GPU), in the benchmark's launch
configuration: one batch of 64 solves run to rel tol 1e-7 on the FP64, the
mixed and the refined mixed paths.

Checks: the GPU set-up pipeline's blocks and step sizes against the CPU
generator on seeded solves; a seeded sample of the batch against the FP64
oracle's parareal at the same iteration (FP64 1e-10, mixed 1e-6, FP64
iteration counts equal to the oracle's); every solve of the batch on the
mixed paths against the FP64 path (1e-6)."""
import numpy as np
import pytest
import torch

import oracle.scheme as S
from problem.batch import cpu_problem, gpu_problem, solve_spec

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-6
KEYS = ("M11", "M12", "M22", "A11", "A12", "A22")


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _host(p):
    out = {k: p[k].cpu().numpy() for k in KEYS}
    out.update(G=p["G"].cpu().numpy(), H=p["H"], time_mode=1, N=p["N"], P=p["P"], dt=p["dt"],
               dt_fine=p["dt_fine"])
    return out


@pytest.mark.parametrize("b", [3, 11])
def test_batch_solve_spaces_match_cpu_generator(b):
    """Solve b's set-up on the GPU against the CPU generator: the local
    eigenvalues of eq. (3.1) (every element); given the CPU's local spectral
    data, the basis functions of eq. (3.2) and the blocks and source factors
    of eq. (3.8); and the stable step computed from those blocks. (On the
    channel-free elements the local eigenvalues are multiple, so the
    eigenvectors each solver picks, and the spaces built from them, are not
    comparable one to one.)"""
    pe = _pe()
    from problem.batch import J1_LOCAL, J_LOCAL, LAYERS, mode_loads, stable_step
    spec = solve_spec(b)
    c = cpu_problem(spec)
    lam = pe.local_spectral(spec["kappa"], spec["n_c"], J_LOCAL)[0].cpu().numpy()
    e_lam = np.abs(lam - c["lam"]).max() / np.abs(c["lam"]).max()
    assert e_lam < 1e-10, (b, e_lam)
    g = pe.cem_spaces(spec["kappa"], c["spsi"], spec["n_c"], LAYERS, J1_LOCAL,
                      loads=mode_loads(spec["n"], spec["pq"]))
    for k in KEYS + ("G",):
        ref = c[k]
        err = np.linalg.norm(g[k].cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (b, k, err)
    _, _, dt_max = stable_step(g["M11"], g["M12"], g["M22"], g["A22"])
    assert abs(0.5 * dt_max - c["dt"]) <= 1e-8 * c["dt"], (0.5 * dt_max, c["dt"])


@pytest.fixture(scope="module")
def batch64():
    pe = _pe()
    probs = [gpu_problem(solve_spec(b)) for b in range(64)]
    print(f"batch of {len(probs)} solves built on the GPU", flush=True)
    out = {}
    for prec in ("fp64", "mixed", "mixed_refine"):
        prs = []
        for p in probs:
            pr = pe.Problem({k: p[k] for k in KEYS}, p["dt"], p["dt_fine"], p["N"], precision=prec)
            pr.set_source(p["G"], p["H"], "interval")
            prs.append(pr)
        bt = pe.Batch(prs)
        x0s = [torch.zeros((1, pr.D), dtype=torch.float64, device="cuda") for pr in prs]
        Xs, its, st = bt.solve(x0s, tol=1e-7, norm="rel")
        assert st == 0
        out[prec] = ([X[0].cpu().numpy() for X in Xs], np.array([int(i[0]) for i in its]))
        print(f"{prec}: batch solved, iterations mean {out[prec][1].mean():.2f}", flush=True)
        bt.close()
        for pr in prs:
            pr.close()
        del Xs
        torch.cuda.empty_cache()
    return probs, out


def test_batch64_sample_against_oracle(batch64):
    probs, out = batch64
    # a seeded sample the oracle finishes in seconds each (D <= 720, N <= 64)
    rng = np.random.default_rng(5)
    sample = [int(b) for b in rng.permutation(len(probs))
              if probs[b]["d1"] + probs[b]["d2"] <= 720 and probs[b]["N"] <= 64][:4]
    assert len(sample) == 4
    for b in sample:
        p = _host(probs[b])
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        r = S.parareal(bl, src, np.zeros(bl.D), 1e-7, rel=True)
        assert out["fp64"][1][b] == r["K"], (b, out["fp64"][1][b], r["K"])
        for prec, bar in (("fp64", TOL64), ("mixed", TOLMIX), ("mixed_refine", TOLMIX)):
            k = min(int(out[prec][1][b]), r["K"])
            err = S.rel_l2_M(bl, out[prec][0][b], r["X"][k])
            print(f"solve {b} (D={bl.D}, N={bl.N}) {prec}: iterations {out[prec][1][b]} (oracle {r['K']}), "
                  f"rel L2 vs oracle {err:.3e}")
            assert err < bar, (b, prec, err)


def test_batch64_mixed_paths_against_fp64(batch64):
    """Every solve of the batch: both mixed paths against the FP64 path (which
    the sampled oracle comparison pins to 1e-10)."""
    probs, out = batch64
    worst = {}
    for prec in ("mixed", "mixed_refine"):
        errs = []
        for b, p in enumerate(probs):
            M = np.block([[p["M11"].cpu().numpy(), p["M12"].cpu().numpy()],
                          [p["M12"].T.cpu().numpy(), p["M22"].cpu().numpy()]])
            X, Xr = out[prec][0][b], out["fp64"][0][b]
            num = np.einsum("ni,ij,nj->", X - Xr, M, X - Xr)
            den = np.einsum("ni,ij,nj->", Xr, M, Xr)
            errs.append(np.sqrt(num / den))
        worst[prec] = max(errs)
        print(f"{prec}: worst rel L2 vs FP64 path over {len(probs)} solves {worst[prec]:.3e}, iterations "
              f"mean {out[prec][1].mean():.2f} (FP64 {out['fp64'][1].mean():.2f})")
        assert worst[prec] < TOLMIX, (prec, worst[prec])
