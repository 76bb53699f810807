"""The standard-EM baseline that bench.py times against CoFEM (explicit Cholesky factorisations
on the GPU through torch.linalg, FP64) reproduces the exact dense EM oracle: E-step quantities
and the M-step's alpha, on the tiny problem and on ragged tasks with an empty one."""

import numpy as np
import pytest
import torch

import bench
import synth
from oracle import cofem, dense_em

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the same baseline, run over 256 matrices of order 1024 (bench.py "
                            "--dense-em), faulted the GPU inside torch.linalg's batched FP64 "
                            "Cholesky / triangular solve; the cause is not established, so the "
                            "baseline stays off the GPU (it passed here at T*C <= 15, D <= 96)"),
]
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("case", ["tiny", "ragged"])
def test_dense_em_baseline_matches_oracle(case):
    if case == "tiny":
        w = synth.make("tiny")
    else:
        w = synth.make(synth.Config("ragged", T=5, C=3, D=96, N=[40, 0, 96, 7, 130],
                                    sparsity=5, groups=3))
    alpha = w.alpha0
    out = bench.dense_em_iteration(
        torch, torch.from_numpy(w.Phi).to(DEV), w.row_off, torch.from_numpy(w.y).to(DEV),
        w.beta, torch.tensor(alpha, device=DEV), torch.tensor(w.log_pi, device=DEV), budget=1 << 20)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    ref = dense_em.estep(w.phi_list(), b, w.beta, alpha)
    q = cofem.responsibilities(ref["ell"], w.log_pi)
    a_new = dense_em.mstep(ref["mu"], ref["var"], q)
    rel = lambda a, r: float(np.max(np.abs(a - r) / np.maximum(np.abs(r), 1e-300)))
    # ell is relative to max(|ell|, |log det|): an empty task's ell is 0 up to rounding
    ell_scale = np.maximum(np.abs(ref["ell"]), np.abs(ref["logdet"]))
    errs = dict(mu=float(np.max(np.abs(g["mu"] - ref["mu"])) / np.max(np.abs(ref["mu"]))),
                var=rel(g["var"], ref["var"]), logdet=rel(g["logdet"], ref["logdet"]),
                ell=float(np.max(np.abs(g["ell"] - ref["ell"]) / ell_scale)),
                q=float(np.max(np.abs(g["q"] - q))), alpha=rel(g["alpha"], a_new))
    print("\n%s: %s" % (case, errs))
    for k, v in errs.items():
        assert v <= 1e-9, (k, v)
