"""Python front end of the cmtcs library: argument marshalling over the C ABI, nothing else.

Every array is a torch tensor on the current HIP device; its pointer goes straight to the C
functions, and the work runs on torch's current stream.  The EM driver ``fit`` is the outer
loop of Alg. 2: E-step and M-step calls, then the final hard assignment.
"""

import ctypes

import numpy as np
import torch

from . import _lib

MATH = {"f64": _lib.CMTCS_MATH_F64, "f32": _lib.CMTCS_MATH_F32, "mixed": _lib.CMTCS_MATH_MIXED}


def _ptr(x):
    return ctypes.c_void_p(0 if x is None else x.data_ptr())


def _cluster_map(col_cluster, T, R):
    """[T][R] int32 host map from a per-column [R] or per-task [T][R] assignment."""
    cc = np.asarray(col_cluster, dtype=np.int32)
    if cc.shape == (R,):
        cc = np.broadcast_to(cc, (T, R))
    if cc.shape != (T, R):
        raise ValueError("col_cluster must have shape (R,) or (T, R)")
    return np.ascontiguousarray(cc)


def _need(x, dtype, shape, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if x.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, x.dtype))
    if tuple(x.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(x.shape)))
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Cmtcs:
    """One problem {(Phi_t, y_t)}, beta, C on the current device (see include/cmtcs.h).

    phi: [sum N_t][D] float32 device tensor (stacked Phi_t); row_off: T+1 prefix sums of N_t
    (host sequence); y: [sum N_t] float32 device tensor.  math: "f64", "f32" or "mixed"; with
    "mixed" the library stores Phi in ``phi16`` ("bf16" or "f16").

    Partial-Fourier sensing (Sec. 4; ``partial_fourier``): phi is None, ``freq`` is the
    [sum N_t] int32 device tensor of selected frequencies, y the [sum N_t][2] float32 (re, im)
    measurements, D the signal length; FP64 only.
    """

    def __init__(self, phi, row_off, y, beta, C, math="f64", max_rhs=None, max_iters=200,
                 max_K=32, phi16="bf16", freq=None, D=None, phi_resid=None):
        lib = _lib.load()
        self.row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        self.T = len(self.row_off) - 1
        self.C = int(C)
        rows = int(self.row_off[-1])
        self.fourier = freq is not None
        if self.fourier:
            if phi is not None:
                raise ValueError("partial-Fourier problems take no phi")
            self.D = int(D)
            _need(freq, torch.int32, (rows,), "freq")
            _need(y, torch.float32, (rows, 2), "y")
        else:
            self.D = int(phi.shape[1])
            _need(phi, torch.float32, (rows, self.D), "phi")
            _need(y, torch.float32, (rows,), "y")
        self.math = math
        self.vdtype = torch.float64 if math == "f64" else torch.float32
        dtype = _lib.CMTCS_F32
        if math == "mixed":
            dtype = {"bf16": _lib.CMTCS_BF16, "f16": _lib.CMTCS_F16}[phi16]
        if phi_resid is not None:
            _need(phi_resid, torch.float32, (rows, self.D), "phi_resid")
        self.phi, self.y, self.freq, self.phi_resid = phi, y, freq, phi_resid
        self.max_K = int(max_K)
        self.max_iters = int(max_iters)
        self.max_rhs = int(max_rhs if max_rhs is not None else self.C * (self.max_K + 1))
        self.beta = float(beta)
        self.device = y.device
        self._roff = self.row_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        p = _lib.Problem(T=self.T, C=self.C, D=self.D, row_off=self._roff,
                         phi=None if phi is None else phi.data_ptr(),
                         phi_dtype=dtype,
                         phi_resid=None if phi_resid is None else phi_resid.data_ptr(),
                         y=y.data_ptr(), beta=self.beta,
                         math=MATH[math], max_rhs=self.max_rhs, max_iters=self.max_iters,
                         max_K=self.max_K,
                         op=_lib.CMTCS_OP_PARTIAL_FOURIER if self.fourier else _lib.CMTCS_OP_DENSE,
                         freq=None if freq is None else freq.data_ptr())
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(lib.cmtcs_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(stream)))
        self._h = h
        self._stream = stream

    @classmethod
    def partial_fourier(cls, freq, row_off, yc, D, beta, C, **kw):
        """A partial-Fourier problem: Phi_t = Omega_t F (the rows ``freq`` of the unitary DFT),
        complex measurements ``yc`` as [sum N_t][2] (re, im) float32 pairs."""
        return cls(None, row_off, yc, beta, C, freq=freq, D=D, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().cmtcs_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_stream(self):
        if torch.cuda.current_stream(self.device).cuda_stream != self._stream:
            raise RuntimeError("the handle was created on another stream")

    @staticmethod
    def _opts(K=0, fixed_iters=0, tol=1e-6, max_iters=200, seed=1, em_iter=0, probes=None,
              alpha_max=1e10, refine_every=0, graph=False, common_probes=False, precond=False):
        return _lib.Opts(K=K, max_iters=max_iters, fixed_iters=fixed_iters, tol=tol,
                         refine_every=refine_every, seed=seed, em_iter=em_iter,
                         probes=None if probes is None else probes.data_ptr(),
                         alpha_max=alpha_max, graph=int(bool(graph)),
                         common_probes=int(bool(common_probes)), precond=int(bool(precond)))

    def estep(self, alpha, log_pi, K, fixed_iters=0, tol=1e-6, max_iters=200, seed=1,
              em_iter=0, probes=None, stats=False, refine_every=0, graph=False,
              common_probes=False, precond=False):
        """One E-step (Alg. 2 inner loop).  Returns a dict of device tensors.  With
        ``common_probes`` every cluster of a task uses the same generated probes; with
        ``precond`` the solves are Jacobi-preconditioned (see cmtcs_opts_t.precond)."""
        self._check_stream()
        T, C, D, dev = self.T, self.C, self.D, self.device
        _need(alpha, torch.float32, (C, D), "alpha")
        _need(log_pi, torch.float64, (C,), "log_pi")
        if probes is not None:
            _need(probes, torch.int8, (T, C, K, D), "probes")
        out = dict(mu=torch.empty(T, C, D, device=dev), s=torch.empty(T, C, D, device=dev),
                   logdet=torch.empty(T, C, dtype=torch.float64, device=dev),
                   ell=torch.empty(T, C, dtype=torch.float64, device=dev),
                   q=torch.empty(T, C, dtype=torch.float64, device=dev))
        st = None
        if stats:
            R = C * (K + 1)
            out["iters"] = torch.empty(T, R, dtype=torch.int32, device=dev)
            out["status"] = torch.empty(T, R, dtype=torch.uint8, device=dev)
            out["ritz_min"] = torch.empty(T, C, K, dtype=torch.float64, device=dev)
            out["ritz_max"] = torch.empty(T, C, K, dtype=torch.float64, device=dev)
            out["k_eff"] = torch.empty(T, C, dtype=torch.int32, device=dev)
            st = _lib.CgStats(out["iters"].data_ptr(), out["status"].data_ptr(),
                              out["ritz_min"].data_ptr(), out["ritz_max"].data_ptr(),
                              out["k_eff"].data_ptr())
        o = self._opts(K=K, fixed_iters=fixed_iters, tol=tol, max_iters=max_iters, seed=seed,
                       em_iter=em_iter, probes=probes, refine_every=refine_every, graph=graph,
                       common_probes=common_probes, precond=precond)
        _lib.check(_lib.load().cmtcs_estep(
            self._h, _ptr(alpha), _ptr(log_pi), ctypes.byref(o), _ptr(out["mu"]), _ptr(out["s"]),
            _ptr(out["logdet"]), _ptr(out["ell"]), _ptr(out["q"]),
            ctypes.byref(st) if st is not None else None))
        return out

    def mstep(self, mu, s, q, alpha, alpha_max=1e10):
        """alpha update of Eq. (mstep), in place on ``alpha``; returns ``alpha``."""
        self._check_stream()
        T, C, D = self.T, self.C, self.D
        _need(mu, torch.float32, (T, C, D), "mu")
        _need(s, torch.float32, (T, C, D), "s")
        _need(q, torch.float64, (T, C), "q")
        _need(alpha, torch.float32, (C, D), "alpha")
        o = self._opts(alpha_max=alpha_max)
        _lib.check(_lib.load().cmtcs_mstep(self._h, _ptr(mu), _ptr(s), _ptr(q), ctypes.byref(o),
                                           _ptr(alpha)))
        return alpha

    def mstep_pi(self, q, log_pi):
        """Learned cluster weights (the mixture-weight M-step the model of Sec. 2 allows):
        log_pi_c = log((1/T) sum_t q_tc), in place on ``log_pi``; returns ``log_pi``."""
        self._check_stream()
        _need(q, torch.float64, (self.T, self.C), "q")
        _need(log_pi, torch.float64, (self.C,), "log_pi")
        _lib.check(_lib.load().cmtcs_mstep_pi(self._h, _ptr(q), _ptr(log_pi)))
        return log_pi

    def log_likelihood(self, ell, log_pi):
        """Marginal log-likelihood estimate of Sec. 2 from an E-step's ell: the per-task L_t
        [T] and their mean Lhat (a one-element tensor), float64 on the device
        (cmtcs_log_likelihood)."""
        self._check_stream()
        _need(ell, torch.float64, (self.T, self.C), "ell")
        _need(log_pi, torch.float64, (self.C,), "log_pi")
        Lt = torch.empty(self.T, dtype=torch.float64, device=self.device)
        L = torch.empty(1, dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().cmtcs_log_likelihood(self._h, _ptr(ell), _ptr(log_pi), _ptr(Lt),
                                                    _ptr(L)))
        return Lt, L

    def em_iter(self, alpha, log_pi, K, out=None, fixed_iters=0, tol=1e-6, max_iters=200,
                seed=1, em_iter=0, probes=None, alpha_max=1e10, graph=False,
                common_probes=False, precond=False):
        """One EM iteration (Alg. 2): E-step from ``alpha``, then the M-step into ``alpha`` (in
        place).  ``out`` (the dict a previous call returned) is reused for the outputs, so that
        with ``graph`` the recorded iteration replays on the same buffers."""
        self._check_stream()
        T, C, D, dev = self.T, self.C, self.D, self.device
        _need(alpha, torch.float32, (C, D), "alpha")
        _need(log_pi, torch.float64, (C,), "log_pi")
        if probes is not None:
            _need(probes, torch.int8, (T, C, K, D), "probes")
        if out is None:
            out = dict(mu=torch.empty(T, C, D, device=dev), s=torch.empty(T, C, D, device=dev),
                       logdet=torch.empty(T, C, dtype=torch.float64, device=dev),
                       ell=torch.empty(T, C, dtype=torch.float64, device=dev),
                       q=torch.empty(T, C, dtype=torch.float64, device=dev))
        o = self._opts(K=K, fixed_iters=fixed_iters, tol=tol, max_iters=max_iters, seed=seed,
                       em_iter=em_iter, probes=probes, alpha_max=alpha_max, graph=graph,
                       common_probes=common_probes, precond=precond)
        _lib.check(_lib.load().cmtcs_em_iter(
            self._h, _ptr(alpha), _ptr(log_pi), ctypes.byref(o), _ptr(out["mu"]), _ptr(out["s"]),
            _ptr(out["logdet"]), _ptr(out["ell"]), _ptr(out["q"])))
        return out

    def solve(self, alpha, B, col_cluster, fixed_iters=0, tol=1e-6, max_iters=200,
              coefs=False, stats=False, graph=False, precond=False):
        """X[t][j] = A_{t, col_cluster[j]}^-1 B[t][j] by CG (Alg. 1)."""
        self._check_stream()
        T, C, D = self.T, self.C, self.D
        R = int(B.shape[1])
        _need(alpha, torch.float32, (C, D), "alpha")
        _need(B, self.vdtype, (T, R, D), "B")
        cc = _cluster_map(col_cluster, T, R)
        X = torch.empty_like(B)
        steps = fixed_iters if fixed_iters > 0 else max_iters
        g = x = None
        if coefs:
            g = torch.empty(T, R, steps, dtype=torch.float64, device=self.device)
            x = torch.empty(T, R, steps, dtype=torch.float64, device=self.device)
        st = None
        out = dict(X=X)
        if stats:
            out["iters"] = torch.empty(T, R, dtype=torch.int32, device=self.device)
            out["status"] = torch.empty(T, R, dtype=torch.uint8, device=self.device)
            st = _lib.CgStats(out["iters"].data_ptr(), out["status"].data_ptr(), None, None, None)
        o = self._opts(fixed_iters=fixed_iters, tol=tol, max_iters=max_iters, graph=graph,
                       precond=precond)
        _lib.check(_lib.load().cmtcs_solve(
            self._h, _ptr(alpha), R, cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(B),
            _ptr(X), _ptr(g), _ptr(x), ctypes.byref(o),
            ctypes.byref(st) if st is not None else None))
        if coefs:
            out["gamma"], out["xi"] = g, x
        return out

    def apply(self, alpha, V, col_cluster):
        """A V column by column (the operator of Eq. (lin-sys)), on the matrix cores."""
        self._check_stream()
        T, C, D = self.T, self.C, self.D
        R = int(V.shape[1])
        _need(alpha, torch.float32, (C, D), "alpha")
        _need(V, self.vdtype, (T, R, D), "V")
        cc = _cluster_map(col_cluster, T, R)
        AV = torch.empty_like(V)
        _lib.check(_lib.load().cmtcs_apply(self._h, _ptr(alpha), R,
                                           cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _ptr(V), _ptr(AV)))
        return AV

    def rhs(self):
        """b_t = beta Phi_t^T y_t as computed by the library, [T][D]."""
        self._check_stream()
        b = torch.empty(self.T, self.D, dtype=self.vdtype, device=self.device)
        _lib.check(_lib.load().cmtcs_rhs(self._h, _ptr(b)))
        return b

    def grad(self, X, Lam, col_cluster, y_coef):
        """(dalpha [C][D], dphi [rows][D]) from solutions X and adjoint solutions Lam
        (see cmtcs_grad in include/cmtcs.h)."""
        self._check_stream()
        T, C, D = self.T, self.C, self.D
        R = int(X.shape[1])
        _need(X, self.vdtype, (T, R, D), "X")
        _need(Lam, self.vdtype, (T, R, D), "Lam")
        cc = _cluster_map(col_cluster, T, R)
        dalpha = torch.empty(C, D, dtype=torch.float32, device=self.device)
        dphi = torch.empty_like(self.phi)
        _lib.check(_lib.load().cmtcs_grad(self._h, R,
                                          cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          _ptr(X), _ptr(Lam), float(y_coef), _ptr(dalpha),
                                          _ptr(dphi)))
        return dalpha, dphi

    def tiles(self):
        """Output rows per wave tile of the (Phi V, Phi^T W) products in use (negative: the
        LDS-staged kernel with four waves of that many rows per tile)."""
        rows = (ctypes.c_int32 * 2)()
        _lib.check(_lib.load().cmtcs_tiles(self._h, rows))
        return int(rows[0]), int(rows[1])

    def profile(self, enable=None):
        """Kernel timing: enable (True/False) and/or read {name: (total ms, launches)}."""
        flag = -1 if enable is None else int(bool(enable))
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        _lib.check(_lib.load().cmtcs_profile(self._h, flag, ms, n))
        names = ("phi_v", "phit_w", "cg_update")
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}


def apply_noalloc(phi, row_off, beta, C, alpha, V, col_cluster, math="f64"):
    """A V (the operator of Eq. (lin-sys)) through cmtcs_apply_noalloc: no handle, no device
    allocation inside the library (its buffers live in a static per-GPU array)."""
    row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
    T = len(row_off) - 1
    D = int(phi.shape[1])
    R = int(V.shape[1])
    vt = torch.float64 if math == "f64" else torch.float32
    _need(phi, torch.float32, (int(row_off[-1]), D), "phi")
    _need(alpha, torch.float32, (int(C), D), "alpha")
    _need(V, vt, (T, R, D), "V")
    cc = _cluster_map(col_cluster, T, R)
    AV = torch.empty_like(V)
    p = _lib.Problem(T=T, C=int(C), D=D,
                     row_off=row_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     phi=phi.data_ptr(), phi_dtype=_lib.CMTCS_F32, phi_resid=None, y=None,
                     beta=float(beta), math=MATH[math], max_rhs=R, max_iters=1, max_K=0,
                     op=_lib.CMTCS_OP_DENSE, freq=None)
    stream = torch.cuda.current_stream(V.device).cuda_stream
    _lib.check(_lib.load().cmtcs_apply_noalloc(
        ctypes.byref(p), _ptr(alpha), R, cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        _ptr(V), _ptr(AV), ctypes.c_void_p(stream)))
    return AV


def fit(model, alpha0, log_pi, K, n_em, fixed_iters=0, tol=1e-6, max_iters=200, seed=1,
        alpha_max=1e10, probes_fn=None, callback=None, graph=False, learn_pi=False,
        common_probes=False, precond=False, start_iter=0):
    """CoFEM (Alg. 2): n_em iterations of E-step + M-step from alpha0, then a_t = argmax_c q_tc
    (lowest c on ties) and mu_{t, a_t} from the last E-step.  With ``graph`` each iteration is
    one replay of the recorded EM iteration (cmtcs_em_iter), on output buffers reused from one
    iteration to the next; ``callback(it, alpha, out)`` then sees alpha as the E-step used it
    (a copy) and the outputs before the next iteration overwrites them.  With ``learn_pi`` each
    M-step also updates the cluster weights (cmtcs_mstep_pi) on a copy of ``log_pi``, returned
    as "log_pi".  ``common_probes``: every cluster of a task uses the same generated probes.
    ``precond``: Jacobi-preconditioned solves (cmtcs_opts_t.precond).

    Checkpoint and resume: the probes of EM iteration ``it`` depend only on (seed, it), so
    iterations start_iter .. start_iter + n_em - 1 from a saved alpha (and log_pi with
    ``learn_pi``) continue a run exactly; a run of n_em iterations equals one of k followed by
    one of n_em - k with start_iter = k, bit for bit."""
    alpha = alpha0.clone()
    log_pi = log_pi.clone() if learn_pi else log_pi
    out = None
    for it in range(start_iter, start_iter + n_em):
        pr = None if probes_fn is None else probes_fn(it)
        if graph:
            before = alpha.clone() if callback is not None else None
            out = model.em_iter(alpha, log_pi, K, out=out, fixed_iters=fixed_iters, tol=tol,
                                max_iters=max_iters, seed=seed, em_iter=it, probes=pr,
                                alpha_max=alpha_max, graph=True, common_probes=common_probes,
                                precond=precond)
            if callback is not None:
                callback(it, before, out)
            if learn_pi:
                model.mstep_pi(out["q"], log_pi)
            continue
        out = model.estep(alpha, log_pi, K, fixed_iters=fixed_iters, tol=tol,
                          max_iters=max_iters, seed=seed, em_iter=it, probes=pr, graph=graph,
                          common_probes=common_probes, precond=precond)
        if callback is not None:
            callback(it, alpha, out)
        model.mstep(out["mu"], out["s"], out["q"], alpha, alpha_max=alpha_max)
        if learn_pi:
            model.mstep_pi(out["q"], log_pi)
    assign = out["q"].cpu().numpy().argmax(axis=1)        # host: first maximum = lowest c
    recon = torch.stack([out["mu"][t, int(assign[t])] for t in range(model.T)])
    return dict(alpha=alpha, q=out["q"], assign=assign, recon=recon, mu=out["mu"], s=out["s"],
                ell=out["ell"], logdet=out["logdet"], log_pi=log_pi)


class CGSolve(torch.autograd.Function):
    """X = A(alpha, Phi)^-1 B column by column, A_tj = beta Phi_t^T Phi_t + diag(alpha_{c_tj})
    (Eq. (lin-sys)), differentiable in B, alpha and Phi.

    Backward (A is symmetric, so the adjoint system uses the same solver): Lam = A^-1 dL/dX,
    dL/dB = Lam, dL/dalpha and dL/dPhi from cmtcs_grad.  ``phi`` must be the tensor the model
    was built on (the library reads it in place); it is an argument only so that autograd
    routes its gradient."""

    @staticmethod
    def forward(ctx, B, alpha, phi, model, col_cluster, tol, max_iters):
        if phi.data_ptr() != model.phi.data_ptr():
            raise ValueError("phi must be the tensor the model was built on")
        X = model.solve(alpha.detach(), B.detach().contiguous(), col_cluster, tol=tol,
                        max_iters=max_iters)["X"]
        ctx.model, ctx.cc, ctx.tol, ctx.max_iters = model, col_cluster, tol, max_iters
        ctx.save_for_backward(alpha, X)
        return X

    @staticmethod
    def backward(ctx, gX):
        alpha, X = ctx.saved_tensors
        m = ctx.model
        Lam = m.solve(alpha.detach(), gX.contiguous(), ctx.cc, tol=ctx.tol,
                      max_iters=ctx.max_iters)["X"]
        dalpha, dphi = m.grad(X, Lam, ctx.cc, y_coef=0.0)
        return Lam, dalpha, dphi, None, None, None, None


class PosteriorMean(torch.autograd.Function):
    """mu_t = A_{t, c_t}(alpha, Phi_t)^-1 (beta Phi_t^T y_t): the posterior mean of task t under
    cluster c_t (Eq. (estep)), differentiable in alpha and Phi (the right-hand side depends on
    Phi too, hence y_coef = 1 in the gradient)."""

    @staticmethod
    def forward(ctx, alpha, phi, model, cluster, tol, max_iters):
        if phi.data_ptr() != model.phi.data_ptr():
            raise ValueError("phi must be the tensor the model was built on")
        cc = np.asarray(cluster, dtype=np.int32).reshape(model.T, 1)
        B = model.rhs().unsqueeze(1).contiguous()
        X = model.solve(alpha.detach(), B, cc, tol=tol, max_iters=max_iters)["X"]
        ctx.model, ctx.cc, ctx.tol, ctx.max_iters = model, cc, tol, max_iters
        ctx.save_for_backward(alpha, X)
        return X[:, 0, :]

    @staticmethod
    def backward(ctx, gmu):
        alpha, X = ctx.saved_tensors
        m = ctx.model
        Lam = m.solve(alpha.detach(), gmu.unsqueeze(1).contiguous(), ctx.cc, tol=ctx.tol,
                      max_iters=ctx.max_iters)["X"]
        dalpha, dphi = m.grad(X, Lam, ctx.cc, y_coef=1.0)
        return dalpha, dphi, None, None, None, None
