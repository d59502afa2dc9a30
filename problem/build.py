"""Seeded synthetic workloads: fine grid + medium -> CEM-GMsFEM spaces ->
projected blocks (paper eq. (3.8)), source factors and initial states.

This module produces the *inputs* of the parareal hot path. It contains no
time stepping, no propagator, no parareal update and no convergence test.

A source is stored in low-rank form f(x, t) = sum_r g_r(x) h_r(t): the
projected spatial factors G = [Psi1^T b_r ; Psi2^T b_r] (D x R, b_r the load
vector of g_r) and time amplitudes H (B x R x T_len). With time_mode "fine",
T_len = N*P and H[..., m] is the amplitude at the fine time t_{m+1}; with
time_mode "interval", T_len = N and H[..., n] holds on (t_n, t_{n+1}].
"""
import hashlib
import json
import os
import time

import numpy as np
import scipy.linalg as sla

from . import media, nlmc
from .cem import CoarseGrid, cem_basis, local_spectral, split_spaces
from .fem import FineGrid

TIME_FINE = 0
TIME_INTERVAL = 1

# Workloads. "c0".."c4" follow the five stated configurations; the small
# "t*" ones keep CPU tests fast.
CONFIGS = {
    "c0": dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="channels", n_h=3, n_v=3,
               contrast=1e4, seed=0, source="one", u0="zero", N=8, P=16, T=1.0, B=1,
               tol=1e-8),
    "c1": dict(n=200, n_c=20, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
               corr=0.05, n_h=5, n_v=5, contrast=1e6, incl=0.2, seed=1,
               source="sine_exp", u0="zero", N=64, P=64, T=None, B=1),
    "c3": dict(n=200, n_c=20, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
               corr=0.05, n_h=5, n_v=5, contrast=1e6, incl=0.2, seed=1,
               source="elem_interval", u0="zero", N=64, P=64, T=None, B=1, src_seed=3),
    "c4": dict(n=400, n_c=40, layers=2, J1=2, J2=3, medium="channels", n_h=10, n_v=10,
               contrast=1e6, seed=4, source="fourier8_interval", u0="zero", N=256, P=128,
               T=None, B=32, src_seed=4),
    # the 200x200 medium with the NLMC split of Section 3.2 (fracture / matrix functions)
    "c1n": dict(n=200, n_c=20, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
                corr=0.05, n_h=5, n_v=5, contrast=1e6, incl=0.2, seed=1, split="nlmc_fm",
                source="sine_exp", u0="zero", N=64, P=64, T=None, B=1),
    # ill-conditioned implicit solves at a stable step: the NLMC split at
    # fracture contrast 1e10 (fractures = cells above 1e3), where
    # cond(M11/dt_fine + A11) reaches about 2e6 (200x200, P = 32)
    "c1s": dict(n=200, n_c=20, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
                corr=0.05, n_h=5, n_v=5, contrast=1e10, incl=0.2, seed=1, split="nlmc_fm",
                frac_threshold=1e3, source="sine_exp", u0="zero", N=64, P=32, T=None, B=1),
    "c4s": dict(n=400, n_c=40, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
                corr=0.05, n_h=10, n_v=10, contrast=1e10, incl=0.2, seed=4, split="nlmc_fm",
                frac_threshold=1e3, source="sine_exp", u0="zero", N=64, P=32, T=None, B=1),
    # small workloads for tests
    "t0": dict(n=20, n_c=2, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1,
               contrast=1e4, seed=10, source="one", u0="zero", N=6, P=4, T=None, B=1),
    "t1": dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="channels", n_h=2, n_v=2,
               contrast=1e6, seed=11, source="sine_exp", u0="sine2", N=8, P=8, T=None, B=1),
    "t1n": dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="channels", n_h=2, n_v=2,
                contrast=1e6, seed=11, split="nlmc_fm", source="sine_exp", u0="sine2", N=8, P=8,
                T=None, B=1),
    "t1p": dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="channels", n_h=2, n_v=2,
                contrast=1e6, seed=11, split="nlmc", source="sine_exp", u0="sine2", N=8, P=8,
                T=None, B=1),
    "t1s": dict(n=40, n_c=4, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0, corr=0.05,
                n_h=2, n_v=2, contrast=1e10, incl=0.5, seed=11, split="nlmc_fm", frac_threshold=1e3,
                source="sine_exp", u0="sine2", N=8, P=8, T=None, B=1),
    "t2": dict(n=60, n_c=6, layers=2, J1=2, J2=3, medium="lognormal", sigma=1.0,
               corr=0.05, n_h=2, n_v=2, contrast=1e6, incl=0.2, seed=12,
               source="fourier8_interval", u0="zero", N=12, P=8, T=None, B=3, src_seed=12),
}


def make_medium(cfg):
    rng = np.random.default_rng(cfg["seed"])
    n, n_c = cfg["n"], cfg["n_c"]
    if cfg["medium"] == "channels":
        kappa, _, _ = media.straight_channels(n, n_c, cfg["n_h"], cfg["n_v"], cfg["contrast"], rng)
    elif cfg["medium"] == "lognormal":
        kappa = media.lognormal_channels(n, n_c, cfg["sigma"], cfg["corr"], cfg["n_h"],
                                         cfg["n_v"], cfg["contrast"], cfg["incl"], rng)
    else:
        raise ValueError(cfg["medium"])
    return kappa


def build_spaces(cfg, kappa=None, checks=False):
    """Fine grid, coarse grid, and (Psi1, Psi2) for a configuration. The split
    is CEM-GMsFEM's eigen-index split (Section 3.1) by default; cfg["split"]
    = "nlmc" / "nlmc_fm" builds the NLMC spaces of Section 3.2 (fractures =
    cells with kappa >= cfg["frac_threshold"], default sqrt(contrast))."""
    if kappa is None:
        kappa = make_medium(cfg)
    fine = FineGrid(kappa)
    cg = CoarseGrid(fine, cfg["n_c"])
    split = cfg.get("split", "cem")
    if split in ("nlmc", "nlmc_fm"):
        thr = cfg.get("frac_threshold") or float(np.sqrt(cfg["contrast"]))
        regions = nlmc.fracture_regions(cg, thr)
        res = nlmc.nlmc_basis(cg, regions, cfg["layers"], return_checks=checks)
        psis, cres = res if checks else (res, None)
        Psi1, Psi2 = nlmc.nlmc_split(cg, psis, "paper" if split == "nlmc" else "fm")
        info = dict(constraint_residual=(max(cres) if cres else None),
                    fractures=int(sum(len(r[1]) for r in regions)))
        return fine, cg, Psi1, Psi2, info
    J = cfg["J1"] + cfg["J2"]
    lam, psi, spsi = local_spectral(cg, J)
    res = cem_basis(cg, J, cfg["layers"], spsi, return_checks=checks)
    phis, cres = res if checks else (res, None)
    Psi1, Psi2 = split_spaces(cg, phis, cfg["J1"], cfg["J2"])
    info = dict(local_eigs=lam, constraint_residual=(max(cres) if cres else None))
    return fine, cg, Psi1, Psi2, info


def project_blocks(fine, Psi1, Psi2):
    """Galerkin blocks of eq. (3.8), symmetrised."""
    out = {}
    MP1, MP2 = fine.M @ Psi1, fine.M @ Psi2
    AP1, AP2 = fine.A @ Psi1, fine.A @ Psi2
    dense = lambda X: np.asarray(X.todense()) if hasattr(X, "todense") else np.asarray(X)
    out["M11"] = dense(Psi1.T @ MP1)
    out["M22"] = dense(Psi2.T @ MP2)
    out["M12"] = dense(Psi1.T @ MP2)
    out["A11"] = dense(Psi1.T @ AP1)
    out["A22"] = dense(Psi2.T @ AP2)
    out["A12"] = dense(Psi1.T @ AP2)
    for k in ("M11", "M22", "A11", "A22"):
        out[k] = 0.5 * (out[k] + out[k].T)
    return out


def diagnostics(bl, with_cond=True):
    """Quantities behind the stability condition of Section 3.2:
    lambda2 = sup over V_H2 of |v|_a^2/|v|^2, gamma^2 = squared largest
    cosine between V_H1 and V_H2 in L2 (eq. (4.15)), and the largest stable
    coarse step (1 - gamma^2)/lambda2."""
    M11, M12, M22, A22 = bl["M11"], bl["M12"], bl["M22"], bl["A22"]
    d2 = M22.shape[0]
    lam2 = float(sla.eigh(A22, M22, eigvals_only=True, subset_by_index=[d2 - 1, d2 - 1])[0])
    X = sla.solve(M11, M12, assume_a="pos")
    C = M12.T @ X
    C = 0.5 * (C + C.T)
    g2 = float(sla.eigh(C, M22, eigvals_only=True, subset_by_index=[d2 - 1, d2 - 1])[0])
    d = dict(lambda2=lam2, gamma2=g2, dt_max=(1.0 - g2) / lam2)
    if with_cond:
        for k in ("M11", "M22", "A11"):
            ev = np.linalg.eigvalsh(bl[k])
            d["cond_" + k] = float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf")
            d["min_eig_" + k] = float(ev[0])
            d["max_eig_" + k] = float(ev[-1])
    return d


def _source(cfg, fine, Psi1, Psi2, N, P, dt, B, cg):
    D = Psi1.shape[1] + Psi2.shape[1]
    proj = lambda b: np.concatenate([Psi1.T @ b, Psi2.T @ b])
    kind = cfg["source"]
    if kind == "one":
        G = proj(fine.load_smooth(lambda x, y: np.ones_like(x)))[:, None]
        H = np.ones((B, 1, N))
        return G, H, TIME_INTERVAL
    if kind == "sine_exp":
        G = proj(fine.load_smooth(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y)))[:, None]
        t = (np.arange(N * P) + 1) * (dt / P)
        H = np.broadcast_to(np.exp(-t)[None, None, :], (B, 1, N * P)).copy()
        return G, H, TIME_FINE
    if kind == "fourier8_interval":
        rng = np.random.default_rng(cfg["src_seed"])
        pq = rng.integers(1, 5, size=(8, 2))
        G = np.stack([proj(fine.load_smooth(
            lambda x, y, p=p, q=q: np.sin(p * np.pi * x) * np.sin(q * np.pi * y)))
            for p, q in pq], axis=1)
        H = rng.standard_normal((B, 8, N))
        return G, H, TIME_INTERVAL
    if kind == "fourier8_const":
        # 8 modes sin(p pi x) sin(q pi y), (p, q) ~ U{1..4}^2, amplitudes
        # N(0,1) per sample, constant in time
        rng = np.random.default_rng(cfg["src_seed"])
        pq = rng.integers(1, 5, size=(8, 2))
        G = np.stack([proj(fine.load_smooth(
            lambda x, y, p=p, q=q: np.sin(p * np.pi * x) * np.sin(q * np.pi * y)))
            for p, q in pq], axis=1)
        a = rng.standard_normal((B, 8, 1))
        return G, np.repeat(a, N, axis=2), TIME_INTERVAL
    if kind == "elem_interval":
        rng = np.random.default_rng(cfg["src_seed"])
        cols = []
        for e in range(cg.n_elem):
            mask = np.zeros(fine.n * fine.n)
            mask[cg.element_cells(e)] = 1.0
            cols.append(proj(fine.load_cells(mask)))
        G = np.stack(cols, axis=1)
        H = rng.standard_normal((B, cg.n_elem, N))
        return G, H, TIME_INTERVAL
    raise ValueError(kind)


def _initial(cfg, fine, Psi1, Psi2, bl, B):
    D = Psi1.shape[1] + Psi2.shape[1]
    if cfg["u0"] == "zero":
        return np.zeros((B, D))
    if cfg["u0"] == "sine2":
        u0 = fine.nodal(lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y))
        rhs = np.concatenate([Psi1.T @ (fine.M @ u0), Psi2.T @ (fine.M @ u0)])
        Mfull = full_mass(bl)
        x0 = sla.solve(Mfull, rhs, assume_a="pos")
        return np.tile(x0, (B, 1))
    raise ValueError(cfg["u0"])


def full_mass(bl):
    return np.block([[bl["M11"], bl["M12"]], [bl["M12"].T, bl["M22"]]])


def full_stiffness(bl):
    return np.block([[bl["A11"], bl["A12"]], [bl["A12"].T, bl["A22"]]])


def _cache_dir():
    d = os.environ.get("PE_CACHE")
    if not d:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".pe_cache")
    os.makedirs(d, exist_ok=True)
    return d


# version of the generators' arithmetic: part of every cache key, so cached
# workloads from an earlier version are not reused
GENERATOR_VERSION = 2


def cfg_key(cfg):
    return hashlib.sha256(json.dumps({"cfg": cfg, "v": GENERATOR_VERSION}, sort_keys=True).encode()).hexdigest()[:16]


# fields that fix the medium and the multiscale spaces (workloads that differ
# only in source, initial state or time grid share them)
_SPACE_FIELDS = ("n", "n_c", "layers", "J1", "J2", "medium", "sigma", "corr", "n_h", "n_v", "contrast",
                 "incl", "seed", "split", "frac_threshold")
_last_spaces = {}


def _spaces(cfg, checks):
    """build_spaces + blocks + diagnostics, memoised for the last space key
    in this process."""
    skey = cfg_key({k: cfg.get(k) for k in _SPACE_FIELDS})
    if not checks and _last_spaces.get("key") == skey:
        return _last_spaces["val"]
    fine, cg, Psi1, Psi2, info = build_spaces(cfg, checks=checks)
    bl = project_blocks(fine, Psi1, Psi2)
    diag = diagnostics(bl, with_cond=Psi1.shape[1] <= 2000)
    val = (fine, cg, Psi1, Psi2, info, bl, diag)
    _last_spaces.clear()
    if not checks:
        _last_spaces.update(key=skey, val=val)
    return val


def build_problem(name_or_cfg, use_cache=True, keep_spaces=False, verbose=False):
    """Build (or load from cache) a workload. Returns a dict with the blocks,
    source factors, initial states, step sizes and diagnostics."""
    cfg = dict(CONFIGS[name_or_cfg]) if isinstance(name_or_cfg, str) else dict(name_or_cfg)
    key = cfg_key(cfg)
    path = os.path.join(_cache_dir(), f"pe_{key}.npz")
    if use_cache and not keep_spaces and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        prob = {k: z[k] for k in z.files if k != "meta"}
        prob.update(json.loads(str(z["meta"])))
        return prob
    t0 = time.perf_counter()
    fine, cg, Psi1, Psi2, info, bl, diag = _spaces(cfg, keep_spaces)
    N, P, B = cfg["N"], cfg["P"], cfg["B"]
    T = cfg.get("T")
    if T is None or T / N > diag["dt_max"]:
        # stated horizon missing or beyond the stability bound of the coarse
        # step: take half the largest stable coarse step
        T_used = N * 0.5 * diag["dt_max"]
    else:
        T_used = T
    dt = T_used / N
    G, H, mode = _source(cfg, fine, Psi1, Psi2, N, P, dt, B, cg)
    x0 = _initial(cfg, fine, Psi1, Psi2, bl, B)
    prob = dict(bl)
    prob.update(G=G, H=H, x0=x0)
    meta = dict(d1=Psi1.shape[1], d2=Psi2.shape[1], N=N, P=P, B=B, dt=dt, dt_fine=dt / P,
                T=T_used, T_stated=T, time_mode=mode, diag=diag, cfg=cfg, key=key,
                build_seconds=time.perf_counter() - t0)
    h = hashlib.sha256()
    for k in ("M11", "M12", "M22", "A11", "A12", "A22", "G", "H", "x0"):
        h.update(np.ascontiguousarray(prob[k]).tobytes())
    meta["sha256"] = h.hexdigest()
    prob.update(meta)
    if verbose:
        print(f"[problem] {key} d1={meta['d1']} d2={meta['d2']} dt={dt:.3e} "
              f"diag={diag} in {meta['build_seconds']:.1f}s", flush=True)
    if keep_spaces:
        prob.update(fine=fine, cg=cg, Psi1=Psi1, Psi2=Psi2, info=info)
    if use_cache:
        np.savez(path, meta=json.dumps(meta), **{k: prob[k] for k in
                 ("M11", "M12", "M22", "A11", "A12", "A22", "G", "H", "x0")})
    return prob
