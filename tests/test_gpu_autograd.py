"""Differentiation form: gradients of losses through x = A(alpha, Phi)^-1 b computed by the
hand-written adjoint CG (cmtcs_solve on dL/dx, A being symmetric) and cmtcs_grad, behind
torch.autograd.Function.

References: the dense FP64 adjoint of oracle/adjoint.py (itself pinned to central differences
and to dense torch autograd in tests/test_oracle_adjoint.py), dense torch autograd on the CPU in
FP64 (torch.linalg.solve on the explicit A), and central differences of the device forward.
CG runs to tol 1e-13, so solutions are exact to ~1e-8 relative on these systems; gradients
are returned in FP32 (the dtype of alpha and Phi).  Bar: relative 1e-5 in the norm of each
gradient block.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint
from paper_2310_00420_amd import CGSolve, PosteriorMean
from gpu_common import DEV, device_model, alpha_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5
CG = dict(tol=1e-13, max_iters=4000)


def _rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _posterior_mean_grads(w, alpha, math="f64", cg=CG):
    m = device_model(w, math=math, K=0, max_rhs=2, max_iters=cg["max_iters"])
    a = alpha_dev(alpha).requires_grad_(True)
    phi = m.phi.requires_grad_(True)
    mu = PosteriorMean.apply(a, phi, m, w.labels, cg["tol"], cg["max_iters"])
    z = torch.tensor(w.z, device=DEV)
    loss = ((mu - z) ** 2).sum()
    loss.backward()
    return mu.detach().cpu().numpy(), a.grad.cpu().numpy(), phi.grad.cpu().numpy()


def _check_against_oracle(w, alpha, math="f64", cg=CG, check=True):
    mu, da, dphi = _posterior_mean_grads(w, alpha, math, cg)
    Phi = [p.astype(np.float64) for p in w.phi_list()]
    y = [v.astype(np.float64) for v in w.y_list()]
    mu_ref = adjoint.forward(Phi, y, alpha, w.beta, w.labels)
    g = adjoint.backward(Phi, y, alpha, w.beta, w.labels, 2 * (mu_ref - w.z))
    e_mu = _rel(mu, mu_ref)
    e_a = _rel(da, g["dalpha"])
    e_p = _rel(dphi, np.concatenate(g["dPhi"], axis=0))
    print("\n%s %s: mu %.2e dalpha %.2e dPhi %.2e" % (w.cfg.name, math, e_mu, e_a, e_p))
    if check:
        assert e_mu <= TOL and e_a <= TOL and e_p <= TOL
    return e_mu, e_a, e_p


def test_posterior_mean_grads_small():
    """D=64, N=32, T=3, C=2: device adjoint vs the dense oracle adjoint."""
    w = synth.make(synth.Config("diff-small", T=3, C=2, D=64, N=32, sparsity=5, groups=2, K=0))
    _check_against_oracle(w, w.alpha0)


def test_posterior_mean_grads_diff_config():
    """The differentiation configuration: T=16, C=2, D=2048, N=512, 40-sparse signals."""
    w = synth.make("diff")
    _check_against_oracle(w, w.alpha0)


# FP32 CG: the recursive residual keeps falling below FP32's resolution, so a tolerance of 1e-9
# stops it after the true solution error has settled at ~kappa u32.
CG32 = dict(tol=1e-9, max_iters=400)


def test_posterior_mean_grads_f32_diff_shape_well_conditioned():
    """The FP32 path at the differentiation configuration's shape (T=16, D=2048, N=512) with
    beta = 1 and alpha in (1, 2) (condition ~10): mu and both gradients within 1e-5."""
    w = synth.make("diff", sigma=1.0)
    _check_against_oracle(w, w.alpha0 + 1.0, math="f32", cg=CG32)


@pytest.mark.xfail(strict=True, reason="at beta = 1e4 and alpha ~ U(0, 1) (condition ~1e8) "
                   "FP32 rounding alone moves the solutions far beyond 1e-5")
def test_posterior_mean_grads_f32_diff_config():
    """The differentiation configuration in FP32, against the 1e-5 bar (expected to fail)."""
    w = synth.make("diff")
    _check_against_oracle(w, w.alpha0, math="f32", cg=CG32)


def test_posterior_mean_grads_central_differences():
    """Central differences of the device forward itself (FP64 CG) at D=64, N=32, for entries
    of alpha, with beta = 50 as in the oracle's own central-difference pin (condition ~1e4, so
    the CG residual at tol 1e-13 is far below the difference signal).  The step is
    h = alpha * 2^-8 and the quotient uses the FP32 values actually applied, so what is left is
    the O((h/alpha)^2) truncation."""
    w = synth.make(synth.Config("diff-small", T=3, C=2, D=64, N=32, sparsity=5, groups=2, K=0,
                                sigma=50 ** -0.5))
    _, da, _ = _posterior_mean_grads(w, w.alpha0)
    m = device_model(w, K=0, max_rhs=2, max_iters=CG["max_iters"])
    z = torch.tensor(w.z, device=DEV)

    def loss(alpha):
        mu = PosteriorMean.apply(alpha_dev(alpha), m.phi, m, w.labels, CG["tol"],
                                 CG["max_iters"])
        return float(((mu - z) ** 2).sum())

    worst = 0.0
    for c, d in [(0, 0), (1, 7), (0, 40), (1, 63)]:
        a0 = w.alpha0[c, d]
        ap = w.alpha0.copy(); am = w.alpha0.copy()
        ap[c, d] = np.float32(a0 + a0 * 2.0 ** -8)
        am[c, d] = np.float32(a0 - a0 * 2.0 ** -8)
        fd = (loss(ap) - loss(am)) / (float(ap[c, d]) - float(am[c, d]))
        worst = max(worst, abs(fd - da[c, d]) / max(abs(fd), 1e-12))
        print("\nalpha[%d,%d]=%.4g: fd %.8e adjoint %.8e" % (c, d, a0, fd, da[c, d]))
    print("central differences: worst rel %.2e (tiles %s)" % (worst, m.tiles()))
    assert worst <= 1e-4   # truncation ~ (2^-8)^2 = 1.5e-5 times a modest constant


def test_cg_solve_grads_dense_autograd():
    """Fixed right-hand sides B (two columns per task, clusters per column): gradients in B,
    alpha and Phi of sum(W * X) against dense torch autograd on the CPU in FP64, D=512."""
    w = synth.make(synth.Config("diff-512", T=2, C=2, D=512, N=128, sparsity=5, groups=2, K=0))
    R = 2
    rng = np.random.default_rng(11)
    B = rng.standard_normal((w.T, R, w.cfg.D))
    Wt = rng.standard_normal((w.T, R, w.cfg.D))
    cc = np.array([[0, 1], [1, 1]], np.int32)
    m = device_model(w, K=0, max_rhs=2 * R, max_iters=CG["max_iters"])
    a = alpha_dev(w.alpha0).requires_grad_(True)
    phi = m.phi.requires_grad_(True)
    Bd = torch.tensor(B, device=DEV, requires_grad=True)
    X = CGSolve.apply(Bd, a, phi, m, cc, CG["tol"], CG["max_iters"])
    (X * torch.tensor(Wt, device=DEV)).sum().backward()

    tP = [torch.tensor(w.phi(t), dtype=torch.float64, requires_grad=True) for t in range(w.T)]
    ta = torch.tensor(w.alpha0, dtype=torch.float64, requires_grad=True)
    tB = torch.tensor(B, requires_grad=True)
    loss = 0
    for t in range(w.T):
        for j in range(R):
            A = w.beta * tP[t].T @ tP[t] + torch.diag(ta[cc[t, j]])
            x = torch.linalg.solve(A, tB[t, j])
            loss = loss + (x * torch.tensor(Wt[t, j])).sum()
    loss.backward()
    e_x = _rel(X.detach().cpu().numpy(),
               np.stack([[torch.linalg.solve(w.beta * tP[t].T @ tP[t] + torch.diag(ta[cc[t, j]]),
                                             tB[t, j]).detach().numpy() for j in range(R)]
                         for t in range(w.T)]))
    e_b = _rel(Bd.grad.cpu().numpy(), tB.grad.numpy())
    e_a = _rel(a.grad.cpu().numpy(), ta.grad.numpy())
    e_p = _rel(phi.grad.cpu().numpy(), np.concatenate([p.grad.numpy() for p in tP], axis=0))
    print("\nCGSolve D=512: X %.2e dB %.2e dalpha %.2e dPhi %.2e" % (e_x, e_b, e_a, e_p))
    assert max(e_x, e_b, e_a, e_p) <= TOL
