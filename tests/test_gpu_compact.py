"""Compaction of stopped columns in the CG loop: the operator products multiply only the column
fragments that hold a task's active right-hand sides (stopped columns move behind them).  Every
output column is the same sequence of operations whichever fragment holds it, so the E-step, the
solve and their statistics are bit-identical to the products over every column slot
(CMTCS_COMPACT=0 at create), on problems whose columns stop at very different steps."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, alpha_dev, device_model, log_pi_dev

pytestmark = pytest.mark.gpu

KEYS = ("mu", "s", "logdet", "ell", "q", "iters", "status", "ritz_min", "ritz_max", "k_eff")


def _spread_alpha(w, scale=1e4):
    """Cluster c's alpha is alpha^0 scaled by scale^(1 - c / (C - 1)): the first cluster's
    systems are diagonally dominant and converge in a few steps, the last cluster's run long."""
    C = w.cfg.C
    f = np.array([scale ** (1.0 - c / max(C - 1, 1)) for c in range(C)])
    return (w.alpha0 * f[:, None]).astype(np.float32).astype(np.float64)


def _both(monkeypatch, build, run):
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("CMTCS_COMPACT", flag)
        m = build()
        r = run(m)
        torch.cuda.synchronize()
        out.append({k: v.clone() for k, v in r.items()})
        m.close()
    monkeypatch.delenv("CMTCS_COMPACT", raising=False)
    return out


def _check_spread(iters, min_stopped=16):
    """At least one task has min_stopped columns that stop before its last one (so whole
    fragments are skipped for a while)."""
    it = iters.cpu().numpy()
    early = (it < it.max(axis=1, keepdims=True)).sum(axis=1)
    print("columns stopping before their task's last one: min %d, max %d of %d"
          % (early.min(), early.max(), it.shape[1]))
    assert early.max() >= min_stopped


def _assert_identical(a, b, keys):
    for k in keys:
        if k in a:
            assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_estep_compacted_equals_full(monkeypatch, math):
    """One column group (R = 132 of 144 slots), columns of the first cluster stopping early."""
    w = synth.make("fp32", T=8)
    alpha = _spread_alpha(w)
    kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=3, em_iter=1, stats=True)
    a, b = _both(monkeypatch, lambda: device_model(w, math=math),
                 lambda m: m.estep(alpha_dev(alpha), log_pi_dev(w.log_pi), w.cfg.K, **kw))
    _check_spread(a["iters"])
    _assert_identical(a, b, KEYS)


def test_estep_compacted_two_groups_ragged(monkeypatch):
    """Two column groups (C = 8, K = 32: 264 right-hand sides in 288 slots) and ragged N_t with
    an empty task: positions past the first group's 144 take the second group's tiles, and a
    group whose positions are all stopped is skipped."""
    w = synth.make("batch", T=6, N=[0, 128, 700, 2048, 333, 1024])
    # the first six clusters' systems are dominated by alpha in (1e8, 2e8) (condition number
    # below 2) and stop within a few steps
    fast = (np.arange(w.cfg.C) < w.cfg.C - 2)[:, None]
    alpha = np.where(fast, 1e8 * (1.0 + w.alpha0), w.alpha0).astype(np.float32).astype(np.float64)
    kw = dict(tol=w.cfg.tol, max_iters=120, seed=1, em_iter=0, stats=True)
    a, b = _both(monkeypatch, lambda: device_model(w, max_iters=120),
                 lambda m: m.estep(alpha_dev(alpha), log_pi_dev(w.log_pi), w.cfg.K, **kw))
    # 121 of 264 stopped: every active position lies in the first group
    _check_spread(a["iters"][1:], min_stopped=121)
    _assert_identical(a, b, KEYS)


def test_estep_compacted_graph_and_precond(monkeypatch):
    """The recorded (HIP graph) loop and the Jacobi-preconditioned loop take the same products."""
    w = synth.make("fp32", T=4)
    alpha = _spread_alpha(w)
    for extra in (dict(graph=True, fixed_iters=60), dict(precond=True)):
        kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=2, em_iter=0, stats=True,
                  **extra)
        a, b = _both(monkeypatch, lambda: device_model(w),
                     lambda m: m.estep(alpha_dev(alpha), log_pi_dev(w.log_pi), w.cfg.K, **kw))
        _assert_identical(a, b, KEYS)


def test_solve_compacted_equals_full(monkeypatch):
    """cmtcs_solve on caller right-hand sides of very different scales (columns meet the
    relative tolerance at different steps), with gamma and xi."""
    w = synth.make("fp32", T=3)
    R = 40
    rng = np.random.default_rng(5)
    B = rng.standard_normal((w.T, R, w.cfg.D)) * 10.0 ** rng.uniform(-3, 3, (w.T, R, 1))
    cc = rng.integers(0, w.cfg.C, (w.T, R)).astype(np.int32)
    alpha = _spread_alpha(w)

    def run(m):
        return m.solve(alpha_dev(alpha), torch.tensor(B, device=DEV), cc, tol=1e-8,
                       max_iters=150, coefs=True, stats=True)
    a, b = _both(monkeypatch, lambda: device_model(w, K=0, max_rhs=R, max_iters=150), run)
    _assert_identical(a, b, ("X", "gamma", "xi", "iters", "status"))
