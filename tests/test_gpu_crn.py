"""Common-random-number probes on the device (opts.common_probes): every cluster of a task uses
the probes generated for cluster 0.  A variance-reduction variant, not in the paper."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, device_model, alpha_dev, log_pi_dev
from oracle import cg as ocg, cofem, probes as oprobes

pytestmark = pytest.mark.gpu

KEYS = ("mu", "s", "logdet", "ell", "q")


def test_common_probes_estep_matches_oracle():
    """Tiny workload, fixed 64 CG steps, K = 16: the device E-step with generated shared probes
    equals the one with the shared probes passed explicitly, and that one meets the E-step
    parity bar against the oracle (every entry within max(1e-5, 4 x the oracle's own
    summation-order spread), as for independent probes)."""
    from test_gpu_estep import _run, _assert
    w = synth.make("tiny")
    K, C = w.cfg.K, w.cfg.C
    P = np.repeat(oprobes.rademacher(1, 0, w.T, C, K, w.cfg.D)[:, :1], C, axis=1)
    err, g, ref, sp = _run(w, range(w.T), probes=P)
    print("\ncommon probes vs oracle:", {k: err[k] for k in ("mu", "s", "logdet", "ell")})
    _assert(err, sp)
    m = device_model(w)
    g2 = m.estep(alpha_dev(w.alpha0), log_pi_dev(w.log_pi), K, fixed_iters=w.cfg.fixed_iters,
                 tol=w.cfg.tol, max_iters=w.cfg.max_iters, common_probes=True)
    for k in KEYS:
        assert torch.equal(g[k], g2[k]), k
    oref = cofem.estep(w.phi_list(), cofem.rhs(w.phi_list(), w.y_list(), w.beta), w.beta,
                       w.alpha0, w.log_pi, K, ocg.CGPolicy(fixed_iters=w.cfg.fixed_iters),
                       common_probes=True)
    assert np.array_equal(oref["ell"], ref["ell"])   # the oracle's shared probes are these


@pytest.mark.parametrize("math", ["f64", "f32", "mixed"])
def test_common_probes_equal_shared_explicit_probes(math):
    """The generated shared probes are the cluster-0 probes of the generator: the same E-step
    with those probes passed explicitly to every cluster gives identical results."""
    w = synth.make("tiny")
    K, C = w.cfg.K, w.cfg.C
    m = device_model(w, math=math)
    a, lp = alpha_dev(w.alpha0), log_pi_dev(w.log_pi)
    kw = dict(fixed_iters=w.cfg.fixed_iters, seed=3, em_iter=2)
    if math == "mixed":
        kw["refine_every"] = 8
    g = m.estep(a, lp, K, common_probes=True, **kw)
    P = oprobes.rademacher(3, 2, w.T, C, K, w.cfg.D)
    P = np.repeat(P[:, :1], C, axis=1).astype(np.int8)
    e = m.estep(a, lp, K, probes=torch.tensor(P, device=DEV), **kw)
    for k in KEYS:
        assert torch.equal(g[k], e[k]), k


def test_em_iter_graph_records_the_probe_mode():
    """A recorded EM iteration is re-recorded when common_probes changes, and every replay
    matches step-by-step launches with the same mode bit for bit."""
    w = synth.make("tiny")
    K = w.cfg.K
    res = {}
    for graph in (False, True):
        m = device_model(w)
        a = alpha_dev(w.alpha0)
        lp = log_pi_dev(w.log_pi)
        out = None
        seq = []
        for i, crn in enumerate((False, True, True, False)):
            a.copy_(alpha_dev(w.alpha0))
            out = m.em_iter(a, lp, K, out=out, fixed_iters=w.cfg.fixed_iters, em_iter=i,
                            graph=graph, common_probes=crn)
            seq.append({k: v.clone() for k, v in out.items()} | {"alpha": a.clone()})
        res[graph] = seq
    for i in range(4):
        for k in KEYS + ("alpha",):
            assert torch.equal(res[False][i][k], res[True][i][k]), (i, k)
    assert not torch.equal(res[False][0]["ell"], res[False][1]["ell"])
