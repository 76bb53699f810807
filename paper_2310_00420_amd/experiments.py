"""Clustered multi-task CS against its two special cases (the first experiment of Sec. 4,
Fig. 1(a)), run on the library's kernels.

Three estimators of the signals z_t from (Phi_t, y_t), each a CoFEM fit (Alg. 2):
  * single-task BCS: every task alone, with its own alpha (T = 1, C = 1 per task);
  * multi-task CS: one alpha shared by all tasks (C = 1);
  * clustered multi-task CS: C clusters with cluster-level alphas and pi_c = 1/C.
Each is scored by the normalised error ||z - mu|| / ||z|| over the concatenation of all tasks,
with mu_t the reconstruction Alg. 2 returns.  The paper's settings for its timing experiments
(50 EM iterations, K = 15 probes, U = 50 CG steps) are the defaults.
"""

import time

import numpy as np
import torch

from .api import Cmtcs, fit


def _alpha0(C, D, seed):
    """alpha^0 ~ Uniform(0, 1) per (c, d) (Alg. 2 initialisation), float32, zeros redrawn."""
    rng = np.random.default_rng(seed)
    a = rng.random((C, D)).astype(np.float32)
    while (a == 0).any():
        z = a == 0
        a[z] = rng.random(int(z.sum())).astype(np.float32)
    return a


def _fit(phi, row_off, y, beta, C, alpha0, n_em, K, steps, seed, math, common_probes=False):
    dev = phi.device
    m = Cmtcs(phi, row_off, y, beta, C, math=math, max_iters=steps, max_K=K)
    try:
        log_pi = torch.full((C,), -np.log(C), dtype=torch.float64, device=dev)
        out = fit(m, torch.tensor(alpha0[:C], device=dev), log_pi, K, n_em, fixed_iters=steps,
                  max_iters=steps, seed=seed, common_probes=common_probes)
        return out["recon"].double().cpu().numpy(), out["assign"]
    finally:
        m.close()


def compare_methods(phi, row_off, y, z, beta, C=2, n_em=50, K=15, steps=50, seed=1,
                    init_seed=420, math="f64"):
    """Normalised errors of the three estimators on one problem.

    phi: [sum N_t][D] float32 device tensor; row_off: T+1 host prefix sums; y: [sum N_t] float32
    device tensor; z: [T][D] true signals (host).  Returns a dict with "single", "multi",
    "clustered" errors, the clustered fit's assignments and the wall time of each method, and
    "clustered_common", "assign_common": the clustered fit with probes shared by the clusters
    of a task (common random numbers; not in the paper)."""
    row_off = np.asarray(row_off, np.int64)
    T, D = len(row_off) - 1, int(phi.shape[1])
    z = np.asarray(z, np.float64)
    a0 = _alpha0(max(C, 1), D, init_seed)
    res, times = {}, {}

    def err(mu):
        return float(np.linalg.norm(z - mu) / np.linalg.norm(z))

    t0 = time.perf_counter()
    mu = np.zeros((T, D))
    for t in range(T):
        r0, r1 = int(row_off[t]), int(row_off[t + 1])
        mu[t] = _fit(phi[r0:r1], [0, r1 - r0], y[r0:r1], beta, 1, a0, n_em, K, steps, seed,
                     math)[0][0]
    times["single"] = time.perf_counter() - t0
    res["single"] = err(mu)

    t0 = time.perf_counter()
    res["multi"] = err(_fit(phi, row_off, y, beta, 1, a0, n_em, K, steps, seed, math)[0])
    times["multi"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    mu, assign = _fit(phi, row_off, y, beta, C, a0, n_em, K, steps, seed, math)
    times["clustered"] = time.perf_counter() - t0
    res["clustered"] = err(mu)
    res["assign"] = np.asarray(assign)

    t0 = time.perf_counter()
    mu, assign = _fit(phi, row_off, y, beta, C, a0, n_em, K, steps, seed, math,
                      common_probes=True)
    times["clustered_common"] = time.perf_counter() - t0
    res["clustered_common"] = err(mu)
    res["assign_common"] = np.asarray(assign)
    res["seconds"] = times
    return res
