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
    (host sequence); y: [sum N_t] float32 device tensor.
    """

    def __init__(self, phi, row_off, y, beta, C, math="f64", max_rhs=None, max_iters=200,
                 max_K=32):
        lib = _lib.load()
        self.row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        self.T = len(self.row_off) - 1
        self.D = int(phi.shape[1])
        self.C = int(C)
        rows = int(self.row_off[-1])
        _need(phi, torch.float32, (rows, self.D), "phi")
        _need(y, torch.float32, (rows,), "y")
        self.math = math
        self.vdtype = torch.float64 if math == "f64" else torch.float32
        self.phi, self.y = phi, y
        self.max_K = int(max_K)
        self.max_iters = int(max_iters)
        self.max_rhs = int(max_rhs if max_rhs is not None else self.C * (self.max_K + 1))
        self.beta = float(beta)
        self.device = phi.device
        self._roff = self.row_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        p = _lib.Problem(T=self.T, C=self.C, D=self.D, row_off=self._roff, phi=phi.data_ptr(),
                         phi_dtype=_lib.CMTCS_F32, phi_f32=None, y=y.data_ptr(), beta=self.beta,
                         math=MATH[math], max_rhs=self.max_rhs, max_iters=self.max_iters,
                         max_K=self.max_K)
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(lib.cmtcs_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(stream)))
        self._h = h
        self._stream = stream

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
              alpha_max=1e10, refine_every=0):
        return _lib.Opts(K=K, max_iters=max_iters, fixed_iters=fixed_iters, tol=tol,
                         refine_every=refine_every, seed=seed, em_iter=em_iter,
                         probes=None if probes is None else probes.data_ptr(),
                         alpha_max=alpha_max)

    def estep(self, alpha, log_pi, K, fixed_iters=0, tol=1e-6, max_iters=200, seed=1,
              em_iter=0, probes=None, stats=False):
        """One E-step (Alg. 2 inner loop).  Returns a dict of device tensors."""
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
            st = _lib.CgStats(out["iters"].data_ptr(), out["status"].data_ptr(),
                              out["ritz_min"].data_ptr(), out["ritz_max"].data_ptr())
        o = self._opts(K=K, fixed_iters=fixed_iters, tol=tol, max_iters=max_iters, seed=seed,
                       em_iter=em_iter, probes=probes)
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

    def solve(self, alpha, B, col_cluster, fixed_iters=0, tol=1e-6, max_iters=200,
              coefs=False, stats=False):
        """X[t][j] = A_{t, col_cluster[j]}^-1 B[t][j] by CG (Alg. 1)."""
        self._check_stream()
        T, C, D = self.T, self.C, self.D
        R = int(B.shape[1])
        _need(alpha, torch.float32, (C, D), "alpha")
        _need(B, self.vdtype, (T, R, D), "B")
        cc = np.ascontiguousarray(np.asarray(col_cluster, dtype=np.int32))
        if cc.shape != (R,):
            raise ValueError("col_cluster must have one entry per column")
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
            st = _lib.CgStats(out["iters"].data_ptr(), out["status"].data_ptr(), None, None)
        o = self._opts(fixed_iters=fixed_iters, tol=tol, max_iters=max_iters)
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
        cc = np.ascontiguousarray(np.asarray(col_cluster, dtype=np.int32))
        if cc.shape != (R,):
            raise ValueError("col_cluster must have one entry per column")
        AV = torch.empty_like(V)
        _lib.check(_lib.load().cmtcs_apply(self._h, _ptr(alpha), R,
                                           cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _ptr(V), _ptr(AV)))
        return AV

    def profile(self, enable=None):
        """Kernel timing: enable (True/False) and/or read {name: (total ms, launches)}."""
        flag = -1 if enable is None else int(bool(enable))
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        _lib.check(_lib.load().cmtcs_profile(self._h, flag, ms, n))
        names = ("phi_v", "phit_w", "cg_update")
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}


def fit(model, alpha0, log_pi, K, n_em, fixed_iters=0, tol=1e-6, max_iters=200, seed=1,
        alpha_max=1e10, probes_fn=None, callback=None):
    """CoFEM (Alg. 2): n_em iterations of E-step + M-step from alpha0, then a_t = argmax_c q_tc
    (lowest c on ties) and mu_{t, a_t} from the last E-step."""
    alpha = alpha0.clone()
    out = None
    for it in range(n_em):
        pr = None if probes_fn is None else probes_fn(it)
        out = model.estep(alpha, log_pi, K, fixed_iters=fixed_iters, tol=tol,
                          max_iters=max_iters, seed=seed, em_iter=it, probes=pr)
        if callback is not None:
            callback(it, alpha, out)
        model.mstep(out["mu"], out["s"], out["q"], alpha, alpha_max=alpha_max)
    assign = out["q"].cpu().numpy().argmax(axis=1)        # host: first maximum = lowest c
    recon = torch.stack([out["mu"][t, int(assign[t])] for t in range(model.T)])
    return dict(alpha=alpha, q=out["q"], assign=assign, recon=recon, mu=out["mu"], s=out["s"],
                ell=out["ell"], logdet=out["logdet"])
