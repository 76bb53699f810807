"""Helpers shared by the GPU tests: building a device problem from a synthetic workload and the
error metrics used to compare the HIP path with the FP64 oracle."""

import numpy as np
import torch

import synth
from paper_2310_00420_amd import Cmtcs

DEV = torch.device("cuda:0")


def device_model(w, math="f64", K=None, max_iters=None, max_rhs=None):
    K = w.cfg.K if K is None else K
    steps = w.cfg.fixed_iters if w.cfg.fixed_iters > 0 else w.cfg.max_iters
    max_iters = steps if max_iters is None else max_iters
    phi = torch.from_numpy(np.ascontiguousarray(w.Phi)).to(DEV)
    y = torch.from_numpy(np.ascontiguousarray(w.y)).to(DEV)
    return Cmtcs(phi, w.row_off, y, w.beta, w.cfg.C, math=math, max_iters=max_iters,
                 max_K=K, max_rhs=max_rhs)


def alpha_dev(alpha):
    return torch.tensor(np.asarray(alpha, np.float32), device=DEV)


def log_pi_dev(log_pi):
    return torch.tensor(np.asarray(log_pi, np.float64), device=DEV)


def rel_cols(a, b):
    """max over the leading indices of ||a - b|| / ||b|| along the last axis."""
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    num = np.linalg.norm(a - b, axis=-1)
    den = np.linalg.norm(b, axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def rel_max(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def estep_errors(got, ref):
    """Per-(t, c) errors of one E-step result against another (both as numpy dicts with the
    oracle's keys mu, s, nu, ell, q): relative vector norms for mu and s, and their largest
    entry error relative to the largest entry (mu_inf, s_inf), relative values for nu, and for
    ell relative to max(|ell|, |nu|) (ell itself can be ~0, e.g. for a task without
    measurements, where nu = -sum log alpha exactly)."""
    def cols(a, b):
        a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
        return np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), 1e-300)

    def elems(a, b):
        # largest entry error relative to the largest entry: a localised error (one wrong tile)
        # is not diluted by the vector length as in the norm ratio
        a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
        return np.max(np.abs(a - b), axis=-1) / np.maximum(np.max(np.abs(b), axis=-1), 1e-300)
    ell_scale = np.maximum(np.abs(ref["ell"]), np.abs(ref["nu"]))
    return dict(mu=cols(got["mu"], ref["mu"]), s=cols(got["s"], ref["s"]),
                mu_inf=elems(got["mu"], ref["mu"]), s_inf=elems(got["s"], ref["s"]),
                logdet=np.abs(got["nu"] - ref["nu"]) / np.abs(ref["nu"]),
                ell=np.abs(got["ell"] - ref["ell"]) / ell_scale)


def compare_estep(gpu, ref, tasks):
    """Error metrics of a device E-step against the oracle's on the same tasks: per-(t, c)
    arrays under "per", their maxima, and the argmax agreement of q."""
    g = {k: v.cpu().numpy() for k, v in gpu.items()}
    t = np.asarray(tasks)
    got = dict(mu=g["mu"][t], s=g["s"][t], nu=g["logdet"][t], ell=g["ell"][t])
    per = estep_errors(got, ref)
    # argmax of q is unique only where the top two z = ell/2 + log pi are apart
    z = 0.5 * ref["ell"]
    zs = np.sort(z, axis=1)
    gap = zs[:, -1] - zs[:, -2] if z.shape[1] > 1 else np.full(len(z), np.inf)
    decided = gap > 1e-6 * np.max(np.abs(ref["nu"]), axis=1)
    out = {k: float(np.max(v)) for k, v in per.items()}
    out.update(q_abs=float(np.max(np.abs(g["q"][t] - ref["q"]))),
               argmax_equal=bool(np.all((g["q"][t].argmax(1) == ref["q"].argmax(1))[decided])),
               undecided_tasks=int((~decided).sum()), per=per)
    return out


def kappa_hat(gpu, tasks):
    """Largest ratio of the extreme Ritz values of the probe tridiagonals (stats ritz_min and
    ritz_max) over the given tasks: a lower bound on the condition number of A."""
    t = np.asarray(tasks)
    return float(np.nanmax(gpu["ritz_max"].cpu().numpy()[t] / gpu["ritz_min"].cpu().numpy()[t]))
