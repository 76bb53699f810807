"""cmtcs_apply_noalloc (the operator without a handle, buffers in a static per-GPU array)
against cmtcs_apply on a handle, on two calls in a row, the second with a smaller problem, in
FP64 and FP32; both against the dense FP64 product."""

import numpy as np
import pytest
import torch

import synth
from paper_2310_00420_amd.api import apply_noalloc
from gpu_common import DEV, device_model, alpha_dev

pytestmark = pytest.mark.gpu


def _case(T, D, Ns, R, seed):
    w = synth.make(synth.Config("noalloc", T=T, C=2, D=D, N=list(Ns), sparsity=4, groups=1, K=0))
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((T, R, D))
    cc = rng.integers(0, 2, (T, R)).astype(np.int32)
    return w, V, cc


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_apply_noalloc_matches_apply(math):
    vt = torch.float64 if math == "f64" else torch.float32
    bar = 1e-12 if math == "f64" else 1e-5
    cases = [(_case(3, 96, [40, 0, 70], 20, 1)), (_case(2, 48, [9, 30], 5, 2))]
    for w, V, cc in cases:
        print("case T=%d D=%d R=%d math=%s" % (w.T, w.cfg.D, V.shape[1], math), flush=True)
        m = device_model(w, math=math, K=0, max_rhs=V.shape[1], max_iters=1)
        Vd = torch.tensor(V, dtype=vt, device=DEV)
        a = alpha_dev(w.alpha0)
        ref = m.apply(a, Vd, cc).cpu().numpy().astype(np.float64)
        got = apply_noalloc(m.phi, w.row_off, w.beta, 2, a, Vd, cc, math=math)
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.float64)
        dense = np.stack([w.beta * (w.phi(t).astype(np.float64).T @ (w.phi(t).astype(np.float64)
                                                                     @ V[t].T)).T
                          + w.alpha0[cc[t]] * V[t] for t in range(w.T)])
        e_ref = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        e_dense = np.max(np.abs(got - dense)) / np.max(np.abs(dense))
        print("  vs cmtcs_apply %.2e, vs dense %.2e" % (e_ref, e_dense))
        assert e_ref <= bar and e_dense <= bar
        m.close()
