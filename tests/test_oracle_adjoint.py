"""Pins of the dense adjoint reference (differentiation form) by finite differences and autograd."""

import numpy as np
import torch

import synth
from oracle import adjoint


def _small(D=64, N=32, T=3, C=2, seed=0):
    w = synth.make("tiny", data_seed=seed, T=T, C=C, D=D, N=N, sparsity=5, groups=C)
    return w.phi_list(), w.y_list(), w.alpha0, w.beta, w.labels, w.z


def _loss(Phi, y, alpha, beta, cl, z):
    mu = adjoint.forward(Phi, y, alpha, beta, cl)
    return float(np.sum((mu - z) ** 2)), mu


def test_gradients_match_central_differences():
    Phi, y, alpha, beta, cl, z = _small()
    beta = 50.0
    Phi = [p.astype(np.float64) for p in Phi]; y = [v.astype(np.float64) for v in y]
    L0, mu = _loss(Phi, y, alpha, beta, cl, z)
    g = adjoint.backward(Phi, y, alpha, beta, cl, 2 * (mu - z))
    h = 1e-4                          # central differences: O(h^2) truncation, roundoff ~ eps L / h
    for c, d in [(0, 0), (1, 7), (0, 40)]:
        ap, am = alpha.copy(), alpha.copy()
        ap[c, d] += h; am[c, d] -= h
        fd = (_loss(Phi, y, ap, beta, cl, z)[0] - _loss(Phi, y, am, beta, cl, z)[0]) / (2 * h)
        assert np.isclose(g["dalpha"][c, d], fd, rtol=1e-6, atol=1e-9)
    for t, i, d in [(0, 0, 0), (1, 5, 9), (2, 31, 63)]:
        Pp = [p.copy() for p in Phi]; Pm = [p.copy() for p in Phi]
        Pp[t][i, d] += h; Pm[t][i, d] -= h
        fd = (_loss(Pp, y, alpha, beta, cl, z)[0] - _loss(Pm, y, alpha, beta, cl, z)[0]) / (2 * h)
        assert np.isclose(g["dPhi"][t][i, d], fd, rtol=1e-6, atol=1e-8)
    for t, i in [(0, 3), (2, 17)]:
        yp = [v.copy() for v in y]; ym = [v.copy() for v in y]
        yp[t][i] += h; ym[t][i] -= h
        fd = (_loss(Phi, yp, alpha, beta, cl, z)[0] - _loss(Phi, ym, alpha, beta, cl, z)[0]) / (2 * h)
        assert np.isclose(g["dy"][t][i], fd, rtol=1e-6, atol=1e-9)


def test_gradients_match_dense_autograd():
    Phi, y, alpha, beta, cl, z = _small(D=512, N=128, T=2, C=2, seed=3)
    mu = adjoint.forward(Phi, y, alpha, beta, cl)
    g = adjoint.backward(Phi, y, alpha, beta, cl, 2 * (mu - z))
    tP = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in Phi]
    ty = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in y]
    ta = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    loss = 0
    for t in range(len(tP)):
        A = beta * tP[t].T @ tP[t] + torch.diag(ta[cl[t]])
        m = torch.linalg.solve(A, beta * tP[t].T @ ty[t])
        loss = loss + ((m - torch.tensor(z[t])) ** 2).sum()
    loss.backward()
    assert np.allclose(ta.grad.numpy(), g["dalpha"], rtol=1e-7, atol=1e-10 * np.abs(g["dalpha"]).max())
    for t in range(len(tP)):
        assert np.allclose(tP[t].grad.numpy(), g["dPhi"][t], rtol=1e-7, atol=1e-10 * np.abs(g["dPhi"][t]).max())
        assert np.allclose(ty[t].grad.numpy(), g["dy"][t], rtol=1e-7, atol=1e-9 * np.abs(g["dy"][t]).max())
