"""The matrix-core operator products and the batched CG against FP64 references.

apply: A V = beta Phi_t^T (Phi_t V) + alpha_{c(j)} (.) V (Eq. (lin-sys), Sec. 3.3), compared with
the same product in FP64 numpy.  Bounds: FP64 arithmetic, relative 1e-12 per column; FP32
arithmetic, relative 1e-5 per column (a few hundred FP32 roundings of non-cancelling sums).
solve: Alg. 1 against the oracle's CG on the same right-hand sides, including the recorded
gamma_u and xi_u.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import cg as ocg
from gpu_common import DEV, device_model, alpha_dev, rel_cols

pytestmark = pytest.mark.gpu


def _ref_apply(w, alpha, V, cc):
    out = np.zeros_like(V, dtype=np.float64)
    for t in range(w.T):
        P = w.phi(t).astype(np.float64)
        for j in range(V.shape[1]):
            v = V[t, j].astype(np.float64)
            out[t, j] = w.beta * (P.T @ (P @ v)) + alpha[cc[j]] * v
    return out


@pytest.mark.parametrize("math,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("shape", [
    dict(T=3, C=2, D=64, N=32, R=5),                       # one tile, padded columns
    dict(T=4, C=3, D=208, N=[0, 17, 70, 129], R=37),      # ragged rows, partial tiles
    dict(T=2, C=4, D=512, N=256, R=150),                   # two column groups
    dict(T=4, C=1, D=48, N=[5, 16, 33, 1], R=9),           # one-chunk tasks, odd chunk count
    dict(T=3, C=2, D=96, N=[40, 0, 23], R=130),            # last fragment 2/16 full, empty task
    # FP32: the forward contraction split over four waves unevenly (25 chunks: 6, 6, 6, 7)
    dict(T=3, C=2, D=400, N=[0, 45, 130], R=21),
])
def test_apply(math, tol, shape):
    shape = dict(shape)
    R = shape.pop("R")
    w = synth.make(synth.Config("op", sparsity=3, groups=1, K=1, **shape))
    m = device_model(w, math=math, K=0, max_rhs=R)
    rng = np.random.default_rng(1)
    V = rng.standard_normal((w.T, R, w.cfg.D))
    cc = rng.integers(0, w.cfg.C, R)
    alpha = w.alpha0
    dt = torch.float64 if math == "f64" else torch.float32
    Vd = torch.tensor(V, dtype=dt, device=DEV)
    got = m.apply(alpha_dev(alpha), Vd, cc).cpu().numpy()
    ref = _ref_apply(w, alpha, Vd.cpu().numpy().astype(np.float64), cc)
    err = rel_cols(got, ref)
    print("\napply %s %s: rel %.2e" % (math, dict(shape, R=R), err))
    assert err <= tol


@pytest.mark.parametrize("math,tol,tiles", [
    ("f64", 1e-12, "32,32"), ("f64", 1e-12, "16,16"), ("f64", 1e-12, "-16,32"),
    ("f64", 1e-12, "-16,16"), ("f64", 1e-12, "-16,-16"), ("f64", 1e-12, "32,-16"),
    ("f32", 1e-5, "64,64"), ("f32", 1e-5, "32,32"), ("f32", 1e-5, "64,-32"),
    ("f32", 1e-5, "32,-32"), ("f32", 1e-5, "16,64"), ("f32", 1e-5, "16,-32")])
@pytest.mark.parametrize("shape", [
    dict(T=4, C=3, D=208, N=[0, 17, 70, 129], R=37),      # ragged rows, partial tiles
    dict(T=2, C=4, D=512, N=[256, 200], R=150),            # two column groups
    dict(T=2, C=4, D=256, N=[96, 40], R=132),              # the measured workload's 132 columns
    dict(T=2, C=3, D=128, N=[64, 33], R=275),              # two groups, last fragment 3/16 full
])
def test_apply_every_tile_shape(math, tol, tiles, shape, monkeypatch):
    """Every tile shape of both products (pinned through CMTCS_TILES), including the LDS-staged
    kernels, whose four-wave tiles run past the rows of small tasks, and column counts
    whose last 16-column fragment is mostly padding (R = 132, 275)."""
    monkeypatch.setenv("CMTCS_TILES", tiles)
    shape = dict(shape)
    R = shape.pop("R")
    w = synth.make(synth.Config("op", sparsity=3, groups=1, K=1, **shape))
    m = device_model(w, math=math, K=0, max_rhs=R)
    assert [int(v) for v in tiles.split(",")] == list(m.tiles())
    rng = np.random.default_rng(4)
    V = rng.standard_normal((w.T, R, w.cfg.D))
    cc = rng.integers(0, w.cfg.C, R)
    dt = torch.float64 if math == "f64" else torch.float32
    Vd = torch.tensor(V, dtype=dt, device=DEV)
    got = m.apply(alpha_dev(w.alpha0), Vd, cc).cpu().numpy()
    ref = _ref_apply(w, w.alpha0, Vd.cpu().numpy().astype(np.float64), cc)
    err = rel_cols(got, ref)
    print("\napply %s tiles %s %s: rel %.2e" % (math, tiles, dict(shape, R=R), err))
    assert err <= tol


def test_solve_matches_oracle_cg():
    """cmtcs_solve on the tiny problem with random right-hand sides, fixed 20 steps: X, gamma_u
    and xi_u against Alg. 1 in FP64.  At 20 of D = 64 steps CG is still far from its
    loss-of-orthogonality regime (the oracle's own summation-order spread is ~1e-11 here; past
    ~25 steps it grows to O(1) on these condition-1e8 systems), so the bar is 1e-8."""
    w = synth.make("tiny")
    C, D = w.cfg.C, w.cfg.D
    R = 6
    rng = np.random.default_rng(3)
    B = rng.standard_normal((w.T, R, D))
    cc = np.array([0, 1, 0, 1, 1, 0])
    m = device_model(w, K=0, max_rhs=R, max_iters=20)
    out = m.solve(alpha_dev(w.alpha0), torch.tensor(B, device=DEV), cc, fixed_iters=20,
                  coefs=True, stats=True)
    X = out["X"].cpu().numpy()
    g = out["gamma"].cpu().numpy()
    x = out["xi"].cpu().numpy()
    ex = eg = exi = 0.0
    for t in range(w.T):
        P = w.phi(t).astype(np.float64)
        acol = np.stack([w.alpha0[c] for c in cc], axis=1)

        def apply_A(V, cols, P=P, acol=acol):
            return w.beta * (P.T @ (P @ V)) + acol[:, cols] * V

        Xo, go, xo, it, st = ocg.cg(apply_A, B[t].T, ocg.CGPolicy(fixed_iters=20))
        ex = max(ex, rel_cols(X[t], Xo.T))
        for j in range(R):
            n = len(go[j])
            assert out["iters"][t, j].item() == n
            eg = max(eg, float(np.max(np.abs(g[t, j, :n] - go[j]) / np.abs(go[j]))))
            exi = max(exi, float(np.max(np.abs(x[t, j, :n] - xo[j]) / np.abs(xo[j]))))
            assert np.all(g[t, j, n:] == 0)
    print("\nsolve: X rel %.2e, gamma rel %.2e, xi rel %.2e" % (ex, eg, exi))
    assert ex <= 1e-8 and eg <= 1e-8 and exi <= 1e-8
