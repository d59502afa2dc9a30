"""Python binding of libpe: argument marshalling only. Every step of the
parareal path runs in the library's HIP kernels; torch provides device
memory and the stream."""
import ctypes

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(x, device):
    t = torch.as_tensor(x, dtype=torch.float64)
    return t.to(device).contiguous()


class Problem:
    """One multiscale problem: blocks of eq. (3.8) + step sizes + N.

    blocks: dict with M11, M22, A11, A12, A22 and optionally M12, A21 (numpy
    arrays or tensors, FP64). precision: "fp64", "mixed" or "mixed_refine"."""

    def __init__(self, blocks, dt, dt_fine, N, precision="fp64", device="cuda", stream=None):
        self.lib = L.load()
        self.device = torch.device(device)
        self.d1 = int(blocks["M11"].shape[0])
        self.d2 = int(blocks["M22"].shape[0])
        self.D = self.d1 + self.d2
        self.N = int(N)
        self.dt, self.dt_fine = float(dt), float(dt_fine)
        self.precision = precision
        prec = {"fp64": L.PE_FP64, "mixed": L.PE_MIXED, "mixed_refine": L.PE_MIXED_REFINE}[precision]
        # a stream of the problem's own (default priority), ordered after the
        # caller's current stream at every call; every library call blocks
        # until its work is done, so results are ready when it returns
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        t = {k: _dev(v, self.device) for k, v in blocks.items() if v is not None}
        self._order()
        h = ctypes.c_void_p()
        st = L.check(self.lib.pe_problem_create(
            ctypes.byref(h), self.d1, self.d2, _ptr(t["M11"]), _ptr(t.get("M12")), _ptr(t["M22"]),
            _ptr(t["A11"]), _ptr(t["A12"]), _ptr(t.get("A21")), _ptr(t["A22"]), self.dt,
            self.dt_fine, self.N, prec, ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h
        P = ctypes.c_int()
        self.lib.pe_problem_info(h, None, None, None, ctypes.byref(P))
        self.P = P.value
        self.B = None
        self.carry = False

    def _order(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def set_source(self, G, H, time_mode):
        """G: D x R projected spatial factors, H: B x R x T_len amplitudes."""
        G = None if G is None else _dev(G, self.device)
        H = None if H is None else _dev(H, self.device)
        self._order()
        R = 0 if G is None else int(G.shape[1])
        B = 1 if H is None else int(H.shape[0])
        mode = {"fine": L.PE_T_FINE, "interval": L.PE_T_INTERVAL, 0: L.PE_T_FINE,
                1: L.PE_T_INTERVAL}[time_mode]
        L.check(self.lib.pe_source_set(self.handle, B, R, _ptr(G), _ptr(H), mode))
        self.B = B
        self.R = R
        self.time_mode = mode
        self.T_len = self.N * self.P if mode == L.PE_T_FINE else self.N
        self._src_keep = (G, H)

    @property
    def S(self):
        """Entries per state: D, or 2D ([x; delta]) with carried history."""
        return 2 * self.D if self.carry else self.D

    def set_history(self, mode):
        """"restart" (fresh history at every interval start) or "carry" (the
        state carries its change over the last fine step: states [x; delta]
        of 2D entries in solve, fine and coarse)."""
        m = {"restart": 0, "carry": 1}[mode]
        L.check(self.lib.pe_set_history(self.handle, m))
        self.carry = m == 1

    def solve(self, x0, tol, norm="abs", k_max=None, out=None):
        """Parareal to the stopping test. Returns (X (B, N+1, S) tensor,
        iters (B,) numpy, jump history (B, k_max) numpy, status); S = D, or
        2D with carried history."""
        x0 = _dev(x0, self.device).reshape(-1, self.D)
        B = x0.shape[0]
        k_max = self.N if k_max is None else int(k_max)
        X = out if out is not None else torch.empty((B, self.N + 1, self.S), dtype=torch.float64,
                                                   device=self.device)
        iters = np.zeros(B, dtype=np.int32)
        hist = np.zeros((B, max(k_max, 1)), dtype=np.float64)
        mode = {"abs": L.PE_NORM_M_ABS, "rel": L.PE_NORM_M_REL}[norm]
        self._order()
        st = L.check(self.lib.pe_solve(self.handle, B, _ptr(x0), float(tol), mode, k_max, _ptr(X),
                                       iters.ctypes.data_as(ctypes.c_void_p),
                                       hist.ctypes.data_as(ctypes.c_void_p)))
        return X, iters, hist[:, :k_max], st

    def adjoint(self, Xbar=None, beta=0.0, Ybnd=None, dH=None, tol=0.0, k_max=None, lam=False):
        """Transposed parareal (pe_adjoint). Xbar: (B, N+1, D) cotangents at
        the coarse boundaries; beta, Ybnd (B, N+1, D), dH (B, R, T_len): the
        fine-step tracking term. Returns dict with x0bar (B, D), Hbar
        (B, R, T_len) or None, lam (B, N+1, D) or None, iters, hist, status."""
        Xbar = None if Xbar is None else _dev(Xbar, self.device).reshape(-1, self.N + 1, self.D)
        Ybnd = None if Ybnd is None else _dev(Ybnd, self.device).reshape(-1, self.N + 1, self.D)
        dH = None if dH is None else _dev(dH, self.device)
        B = Xbar.shape[0] if Xbar is not None else (Ybnd.shape[0] if Ybnd is not None else (self.B or 1))
        k_max = self.N if k_max is None else int(k_max)
        x0bar = torch.empty((B, self.D), dtype=torch.float64, device=self.device)
        R = getattr(self, "R", 0)
        Hbar = torch.empty((B, R, self.T_len), dtype=torch.float64, device=self.device) if R else None
        Lam = torch.empty((B, self.N + 1, self.D), dtype=torch.float64, device=self.device) if lam else None
        iters = np.zeros(B, dtype=np.int32)
        hist = np.zeros((B, max(k_max, 1)), dtype=np.float64)
        self._order()
        st = L.check(self.lib.pe_adjoint(self.handle, B, _ptr(Xbar), float(beta), _ptr(Ybnd), _ptr(dH),
                                         float(tol), k_max, _ptr(x0bar), _ptr(Hbar), _ptr(Lam),
                                         iters.ctypes.data_as(ctypes.c_void_p),
                                         hist.ctypes.data_as(ctypes.c_void_p)))
        return dict(x0bar=x0bar, Hbar=Hbar, lam=Lam, iters=iters, hist=hist[:, :k_max], status=st)

    def tracking(self, Ybnd, dH=None, beta=1.0):
        """J_b = 1/2 beta sum_m dt_fine |y_m|_M^2 over the fine levels of the
        trajectory with boundary states Ybnd and source amplitudes dH."""
        Ybnd = _dev(Ybnd, self.device).reshape(-1, self.N + 1, self.D)
        dH = None if dH is None else _dev(dH, self.device)
        J = np.zeros(Ybnd.shape[0])
        self._order()
        L.check(self.lib.pe_tracking(self.handle, Ybnd.shape[0], _ptr(Ybnd), _ptr(dH), float(beta),
                                     J.ctypes.data_as(ctypes.c_void_p)))
        return J

    def fine(self, Xin):
        """F applied to Xin (B, N, S) -> (B, N, S)."""
        Xin = _dev(Xin, self.device)
        B = Xin.shape[0]
        Y = torch.empty_like(Xin)
        self._order()
        L.check(self.lib.pe_fine_propagate(self.handle, B, _ptr(Xin), _ptr(Y)))
        return Y

    def set_fine_solver(self, kind="step", alpha=0.05, K0=1):
        """The fine propagator used by solve(): "step" (P steps of the scheme)
        or "wr" (K0 waveform-relaxation iterations with alpha, FP64 handles)."""
        k = {"step": 0, "wr": 1}[kind]
        L.check(self.lib.pe_set_fine_solver(self.handle, k, float(alpha), int(K0)))

    def fine_wr(self, Xin, alpha, K0):
        """The fine propagator by waveform relaxation with the alpha-circulant
        diagonalisation (K0 iterations, FP64) applied to Xin (B, N, D) ->
        (B, N, D); its fixed point is `fine`."""
        Xin = _dev(Xin, self.device).reshape(-1, self.N, self.D)
        B = Xin.shape[0]
        Y = torch.empty_like(Xin)
        self._order()
        L.check(self.lib.pe_fine_wr(self.handle, B, _ptr(Xin), float(alpha), int(K0), _ptr(Y)))
        return Y

    def coarse(self, Xin):
        """G applied to Xin (B, N, S) -> (B, N, S)."""
        Xin = _dev(Xin, self.device)
        B = Xin.shape[0]
        Y = torch.empty_like(Xin)
        self._order()
        L.check(self.lib.pe_coarse_propagate(self.handle, B, _ptr(Xin), _ptr(Y)))
        return Y

    def coarse_noalloc(self, Xin, Y):
        """G applied to Xin (B, N, D) into the caller's Y, with the library's
        static workspace (pe_coarse_propagate_noalloc: no device allocation)."""
        self._order()
        L.check(self.lib.pe_coarse_propagate_noalloc(self.handle, int(Xin.shape[0]), _ptr(Xin), _ptr(Y)))
        return Y

    def mass_norms(self, X):
        X = _dev(X, self.device).reshape(-1, self.D)
        out = np.zeros(X.shape[0])
        self._order()
        L.check(self.lib.pe_mass_norms(self.handle, X.shape[0], _ptr(X),
                                       out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def autotune(self, B=None):
        """Time candidate tile configurations for the fine sweep (B samples)."""
        self._order()
        L.check(self.lib.pe_autotune(self.handle, int(B or self.B or 1)))

    def profile(self, enable=True):
        """Enable/disable per-launch HIP-event timing (resets totals)."""
        L.check(self.lib.pe_profile(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{kind: (total GPU ms, launches)} since the last profile() call."""
        out = {}
        for name, k in L.PROFILE_KINDS.items():
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            L.check(self.lib.pe_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def last_tiles(self, kind="fine_step"):
        """(state-tile rows, operator-tile rows, K depth, split-K) of the last
        launch of a product class."""
        out = (ctypes.c_int * 4)()
        L.check(self.lib.pe_last_tiles(self.handle, L.PROFILE_KINDS[kind], out))
        return tuple(out)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pe_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Different problems (sizes, interval counts, sources; same precision
    and step ratio) solved together by grouped launches (pe_batch_*). The
    problems must outlive the batch."""

    def __init__(self, problems, device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.problems = list(problems)
        self.stream = torch.cuda.Stream(device=self.device)
        arr = (ctypes.c_void_p * len(self.problems))(*[p.handle.value for p in self.problems])
        h = ctypes.c_void_p()
        L.check(self.lib.pe_batch_create(ctypes.byref(h), len(self.problems), arr,
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h

    def solve(self, x0s, tol, norm="abs", k_max=None):
        """x0s: one (B_i, D_i) initial-state array per problem. Returns
        (list of X_i (B_i, N_i+1, D_i), list of iteration arrays, status)."""
        x0s = [_dev(x, self.device).reshape(-1, p.D) for x, p in zip(x0s, self.problems)]
        Xs = [torch.empty((x.shape[0], p.N + 1, p.D), dtype=torch.float64, device=self.device)
              for x, p in zip(x0s, self.problems)]
        nb = [x.shape[0] for x in x0s]
        k_max = max(p.N for p in self.problems) if k_max is None else int(k_max)
        iters = np.zeros(sum(nb), dtype=np.int32)
        xa = (ctypes.c_void_p * len(x0s))(*[x.data_ptr() for x in x0s])
        Xa = (ctypes.c_void_p * len(Xs))(*[X.data_ptr() for X in Xs])
        mode = {"abs": L.PE_NORM_M_ABS, "rel": L.PE_NORM_M_REL}[norm]
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        st = L.check(self.lib.pe_batch_solve(self.handle, xa, float(tol), mode, k_max, Xa,
                                             iters.ctypes.data_as(ctypes.c_void_p)))
        off = np.cumsum([0] + nb)
        return Xs, [iters[off[i]:off[i + 1]] for i in range(len(nb))], st

    def profile(self, enable=True):
        """Enable/disable per-launch HIP-event timing of the grouped launches."""
        L.check(self.lib.pe_batch_profile(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{kind: (total GPU ms, launches)} since the last profile() call."""
        out = {}
        for name, k in L.PROFILE_KINDS.items():
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            L.check(self.lib.pe_batch_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pe_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_peaks(device="cuda"):
    """Measured peaks of the GPU: {"fp32_mfma_tflops", "fp64_mfma_tflops",
    "hbm_copy_tbps"} (pe_probe_peaks on the device's current stream)."""
    lib = L.load()
    with torch.cuda.device(torch.device(device)):
        out = (ctypes.c_double * 3)()
        L.check(lib.pe_probe_peaks(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), out))
    return {"fp32_mfma_tflops": out[0], "fp64_mfma_tflops": out[1], "hbm_copy_tbps": out[2]}


def local_spectral(kappa, n_c, J, device="cuda"):
    """Local spectral problems of eq. (3.1) on the GPU (pe_local_spectral).
    kappa: (n, n) cell values. Returns device tensors lam (n_c^2, J),
    psi and spsi (n_c^2, (m+1)^2, J)."""
    lib = L.load()
    dev = torch.device(device)
    if torch.is_tensor(kappa):
        kappa = kappa.to(device=dev, dtype=torch.float64).contiguous()
    else:
        kappa = _dev(np.ascontiguousarray(kappa, dtype=np.float64), dev)
    n = kappa.shape[0]
    m = n // n_c
    lam = torch.zeros((n_c * n_c, J), dtype=torch.float64, device=dev)
    psi = torch.zeros((n_c * n_c, (m + 1) ** 2, J), dtype=torch.float64, device=dev)
    spsi = torch.zeros_like(psi)
    with torch.cuda.device(dev):
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        L.check(lib.pe_local_spectral(n, n_c, J, _ptr(kappa), _ptr(lam), _ptr(psi), _ptr(spsi), st))
    return lam, psi, spsi


def cem_spaces(kappa, spsi, n_c, layers, J1, loads=None, want_basis=False, device="cuda", J=None):
    """Multiscale spaces and Galerkin blocks on the GPU (pe_cem_spaces).
    kappa: (n, n) cell values; spsi: (n_c^2, (m+1)^2, J) constraint data of
    the local spectral problems, or None to solve them on the GPU as well
    (pe_local_spectral, J functions per element); loads: (R, (n-1)^2)
    fine-grid load vectors or None. Returns a dict of device tensors M11, M12, M22, A11, A12, A22,
    G (D x R, if loads) and Psi (D x (n-1)^2, if want_basis)."""
    lib = L.load()
    dev = torch.device(device)
    kappa = _dev(np.ascontiguousarray(kappa, dtype=np.float64), dev)
    if spsi is None:
        if J is None:
            raise ValueError("cem_spaces: J (functions per element) is needed when spsi is None")
        _, _, spsi = local_spectral(kappa, n_c, J, device=device)
    else:
        spsi = _dev(np.ascontiguousarray(spsi, dtype=np.float64), dev)
    n = kappa.shape[0]
    n_el, _, J = spsi.shape
    d1, d2 = n_el * J1, n_el * (J - J1)
    D = d1 + d2
    z = lambda r, c: torch.zeros((r, c), dtype=torch.float64, device=dev)
    out = {"M11": z(d1, d1), "M12": z(d1, d2), "M22": z(d2, d2), "A11": z(d1, d1), "A12": z(d1, d2),
           "A22": z(d2, d2)}
    R = 0
    ld = None
    if loads is not None:
        ld = _dev(np.ascontiguousarray(np.atleast_2d(loads), dtype=np.float64), dev)
        R = ld.shape[0]
        out["G"] = z(D, R)
    if want_basis:
        out["Psi"] = z(D, (n - 1) ** 2)
    p = lambda k: _ptr(out[k]) if k in out else None
    with torch.cuda.device(dev):
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        L.check(lib.pe_cem_spaces(n, n_c, layers, J, J1, _ptr(kappa), _ptr(spsi), R,
                                  _ptr(ld) if ld is not None else None, p("M11"), p("M12"), p("M22"),
                                  p("A11"), p("A12"), p("A22"), p("G"), p("Psi"), st))
    return out


def nlmc_spaces(kappa, counts, rdata, n_c, layers, loads=None, want_basis=False, device="cuda"):
    """NLMC spaces split by continuum and their Galerkin blocks on the GPU
    (pe_nlmc_spaces). kappa: (n, n) cell values; counts: regions per coarse
    element (matrix region + fracture pieces); rdata: (n_c^2, (m+1)^2, J)
    region integrals of the local Q1 functions; loads: (R, (n-1)^2) or None.
    Returns a dict of device tensors M11, M12, M22, A11, A12, A22 (V_H1 = the
    fracture functions, V_H2 = the matrix functions), G (if loads) and Psi
    (if want_basis)."""
    lib = L.load()
    dev = torch.device(device)
    kappa = _dev(np.ascontiguousarray(kappa, dtype=np.float64), dev)
    rdata = _dev(np.ascontiguousarray(rdata, dtype=np.float64), dev)
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    n = kappa.shape[0]
    n_el, _, J = rdata.shape
    d1, d2 = int(counts.sum()) - n_el, n_el
    D = d1 + d2
    z = lambda r, c: torch.zeros((r, c), dtype=torch.float64, device=dev)
    out = {"M11": z(d1, d1), "M12": z(d1, d2), "M22": z(d2, d2), "A11": z(d1, d1), "A12": z(d1, d2),
           "A22": z(d2, d2)}
    R = 0
    ld = None
    if loads is not None:
        ld = _dev(np.ascontiguousarray(np.atleast_2d(loads), dtype=np.float64), dev)
        R = ld.shape[0]
        out["G"] = z(D, R)
    if want_basis:
        out["Psi"] = z(D, (n - 1) ** 2)
    p = lambda k: _ptr(out[k]) if k in out else None
    with torch.cuda.device(dev):
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        L.check(lib.pe_nlmc_spaces(n, n_c, layers, J, counts.ctypes.data_as(ctypes.c_void_p), _ptr(kappa),
                                   _ptr(rdata), R, _ptr(ld) if ld is not None else None, p("M11"), p("M12"),
                                   p("M22"), p("A11"), p("A12"), p("A22"), p("G"), p("Psi"), st))
    return out


def problem_from(prob, precision="fp64", device="cuda"):
    """Problem + source from a workload dict (blocks, G, H, time_mode)."""
    blocks = {k: prob[k] for k in ("M11", "M12", "M22", "A11", "A12", "A22")}
    pr = Problem(blocks, prob["dt"], prob["dt_fine"], prob["N"], precision=precision, device=device)
    pr.set_source(prob["G"], prob["H"], int(prob["time_mode"]))
    return pr


class ParaSolve(torch.autograd.Function):
    """X = parareal solution (B, N+1, D) for source amplitudes H (B, R, T_len)
    on the spatial factors G and initial states x0 (B, D). The backward pass
    runs the transposed parareal (pe_adjoint) with dL/dX as the boundary
    cotangents and returns dL/dH and dL/dx0.

    Usage: X = ParaSolve.apply(H, x0, problem, G, time_mode, tol, adj_tol)."""

    @staticmethod
    def forward(ctx, H, x0, problem, G, time_mode, tol, adj_tol):
        problem.set_source(G, H.detach(), time_mode)
        X, _, _, _ = problem.solve(x0.detach(), tol=tol, norm="rel")
        ctx.problem, ctx.adj_tol = problem, adj_tol
        return X

    @staticmethod
    def backward(ctx, dX):
        r = ctx.problem.adjoint(Xbar=dX.contiguous(), tol=ctx.adj_tol)
        return r["Hbar"], r["x0bar"], None, None, None, None, None


class TrackedSolve(torch.autograd.Function):
    """(X, J): the parareal solution for (H, x0) as in ParaSolve, and the
    fine-step tracking term J_b = 1/2 beta sum_{m>=1} dt_fine |x_m - r_m|_M^2
    against the reference trajectory r of (H_ref, x0_ref), given by its
    boundary states X_ref (B, N+1, D). Both terms are differentiated by one
    transposed parareal run.

    Usage: X, J = TrackedSolve.apply(H, x0, problem, G, time_mode, H_ref,
    X_ref, beta, tol, adj_tol)."""

    @staticmethod
    def forward(ctx, H, x0, problem, G, time_mode, H_ref, X_ref, beta, tol, adj_tol):
        problem.set_source(G, H.detach(), time_mode)
        X, _, _, _ = problem.solve(x0.detach(), tol=tol, norm="rel")
        Y = (X - X_ref).contiguous()
        dH = (H.detach() - H_ref).contiguous()
        J = torch.as_tensor(problem.tracking(Y, dH, beta), device=X.device)
        ctx.problem, ctx.adj_tol, ctx.beta = problem, adj_tol, beta
        ctx.save_for_backward(Y, dH)
        return X, J

    @staticmethod
    def backward(ctx, dX, dJ):
        Y, dH = ctx.saved_tensors
        # the tracking term is quadratic in y: its cotangent dJ_b scales y_b
        w = dJ.to(torch.float64).reshape(-1, 1, 1)
        r = ctx.problem.adjoint(Xbar=dX.contiguous(), beta=ctx.beta, Ybnd=(w * Y).contiguous(),
                                dH=(w * dH).contiguous(), tol=ctx.adj_tol)
        return r["Hbar"], r["x0bar"], None, None, None, None, None, None, None, None
