"""The CG loop recorded as one HIP graph (opts.graph) gives bit-identical results to
step-by-step launches: the same kernels in the same order, replayed.  Replays are checked
after eager work between them (an M-step that rewrites alpha in place, whose pointer the
recording keeps), and across several EM iterations."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, device_model, alpha_dev, log_pi_dev
from paper_2310_00420_amd import fit

pytestmark = pytest.mark.gpu

KEYS = ("mu", "s", "logdet", "ell", "q")


def _equal(a, b):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_estep_graph_replays_match_direct(math):
    w = synth.make("fp32", T=8)
    m = device_model(w, math=math)
    alpha = alpha_dev(w.alpha0)
    lp = log_pi_dev(w.log_pi)
    kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=1)
    for it in range(3):                  # record, then replay twice with new probes and alpha
        d = m.estep(alpha, lp, w.cfg.K, em_iter=it, **kw)
        g = m.estep(alpha, lp, w.cfg.K, em_iter=it, graph=True, **kw)
        _equal(d, g)
        m.mstep(g["mu"], g["s"], g["q"], alpha)     # eager work between replays


def test_fit_graph_matches_direct():
    w = synth.make("tiny")
    out = []
    for graph in (False, True):
        m = device_model(w)
        out.append(fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, 4,
                       fixed_iters=w.cfg.fixed_iters, graph=graph))
    assert torch.equal(out[0]["alpha"], out[1]["alpha"])
    assert np.array_equal(out[0]["assign"], out[1]["assign"])
    assert torch.equal(out[0]["mu"], out[1]["mu"])


def test_solve_graph_matches_direct():
    w = synth.make("tiny")
    R = 5
    rng = np.random.default_rng(4)
    B = torch.tensor(rng.standard_normal((w.T, R, w.cfg.D)), device=DEV)
    m = device_model(w, K=0, max_rhs=R, max_iters=30)
    cc = [0, 1, 1, 0, 1]
    d = m.solve(alpha_dev(w.alpha0), B, cc, fixed_iters=30, coefs=True)
    for _ in range(2):
        g = m.solve(alpha_dev(w.alpha0), B, cc, fixed_iters=30, coefs=True, graph=True)
        for k in ("X", "gamma", "xi"):
            assert torch.equal(d[k], g[k]), k


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_em_iter_graph_replays_match_direct(math):
    """cmtcs_em_iter recorded as one graph (E-step and M-step) against cmtcs_estep and
    cmtcs_mstep launched step by step: three EM iterations with new probe keys, and between
    replays a solve with another column count, which rewrites the cluster map and the tile
    tables that the recording reads."""
    w = synth.make("fp32", T=8)
    m = device_model(w, math=math)
    kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=1)
    a_d = alpha_dev(w.alpha0)
    a_g = a_d.clone()
    lp = log_pi_dev(w.log_pi)
    dt = torch.float64 if math == "f64" else torch.float32
    B = torch.tensor(np.random.default_rng(2).standard_normal((w.T, 5, w.cfg.D)), dtype=dt,
                     device=DEV)
    out = None
    for it in range(3):
        d = m.estep(a_d, lp, w.cfg.K, em_iter=it, **kw)
        m.mstep(d["mu"], d["s"], d["q"], a_d)
        out = m.em_iter(a_g, lp, w.cfg.K, out=out, em_iter=it, graph=True, **kw)
        _equal(d, out)
        assert torch.equal(a_d, a_g)
        m.solve(a_g, B, [0, 1, 1, 0, 1], max_iters=20)
