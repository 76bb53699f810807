"""The special cases used by the comparison of Sec. 4, Fig. 1(a): multi-task CS is CoFEM with one
cluster (C = 1) and single-task BCS is CoFEM on one task with its own alpha (T = C = 1)."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, device_model, alpha_dev, log_pi_dev, rel_cols
from oracle import cg as ocg, cofem
from paper_2310_00420_amd import fit

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.mark.parametrize("T", [4, 1])
def test_one_cluster_fit_matches_oracle(T):
    """C = 1 (q is 1 for every task): three EM iterations with converged CG follow the oracle.
    Converged CG, because after a fixed number of unconverged steps the trajectory itself moves
    by ~4e-3 in 1/alpha when alpha^0 moves by 1e-7 (the oracle against itself), the size of the
    device's FP32 rounding of alpha."""
    w = synth.make(synth.Config("c1", T=T, C=1, D=64, N=32, sparsity=6, groups=1, K=16,
                                tol=1e-13, max_iters=640))
    m = device_model(w)
    out = fit(m, alpha_dev(w.alpha0), log_pi_dev([0.0]), w.cfg.K, 3, tol=1e-13, max_iters=640)
    pol = ocg.CGPolicy(tol=1e-13, max_iters=640)
    ref = cofem.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, np.zeros(1), w.cfg.K, pol, 3,
                    seed=1)
    q = out["q"].cpu().numpy()
    e_alpha = rel_cols(1.0 / out["alpha"].cpu().numpy().astype(np.float64), 1.0 / ref["alpha"])
    e_mu = rel_cols(out["mu"].cpu().numpy(), ref["mu"])
    print("\nC=1 T=%d: 1/alpha rel %.2e, mu rel %.2e" % (T, e_alpha, e_mu))
    assert np.all(q == 1.0)
    assert e_alpha <= TOL and e_mu <= TOL


def test_support_difference_orderings():
    """The findings of Fig. 1(a) on Gaussian stand-in sensing matrices (T=8 in two groups of 4,
    D=512, N=D/4, 5% sparsity, sigma=0.05; 50 EM iterations, K=15, U=50): with one common
    support (f=0) sharing alpha beats single-task recovery; with disjoint supports (f=1) one
    shared alpha is no better than single-task recovery, while the clustered model finds the two
    groups and keeps its error low.  Measured: f=0 single 0.096, multi 0.058, clustered 0.062;
    f=1 single 0.105, multi 0.105, clustered 0.069."""
    from paper_2310_00420_amd.experiments import compare_methods
    err = {}
    for f in (0.0, 1.0):
        w = synth.make(synth.Config("support-sweep", T=8, C=2, D=512, N=128, sparsity=26,
                                    groups=2, sigma=0.05, support_diff=f))
        r = compare_methods(torch.from_numpy(w.Phi).to(DEV), w.row_off,
                            torch.from_numpy(w.y).to(DEV), w.z, w.beta, C=2)
        print("\nf=%.1f single %.4f multi %.4f clustered %.4f assign %s"
              % (f, r["single"], r["multi"], r["clustered"], r["assign"]))
        err[f] = r
    e0, e1 = err[0.0], err[1.0]
    assert e0["multi"] < 0.8 * e0["single"] and e0["clustered"] < 0.8 * e0["single"]
    assert e1["clustered"] < 0.8 * e1["multi"] and e1["clustered"] < 0.8 * e1["single"]
    a = e1["assign"]
    assert len(set(a[:4])) == 1 and len(set(a[4:])) == 1 and a[0] != a[4]
