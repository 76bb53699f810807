"""Parity of the HIP E-step and M-step with the FP64 oracle on identical inputs and probes.

Bar: relative 1e-5 on mu, s, nu-bar and ell (per (t, c) vector norm for mu and s; ell relative
to max(|ell|, |nu|)), the bound set for the GPU results against the FP64 oracle, and
identical argmax of q wherever it is decided.

CG on these systems (condition numbers 1e6-1e9) is sensitive to the order of its FP64
roundings once a task's large-eigenvalue cluster is exhausted (Krylov dimension >= rank of
Phi_t, e.g. the tiny problem at U = D = 64 steps, or tasks with N_t << D or N_t ~ D in the
batching configuration): there the oracle itself moves by up to ~5e-4 when only the order of
its sums changes.  Every E-step comparison therefore measures that self-spread -- the oracle
rerun with its operator applied one column at a time, the same arithmetic in another FP64
order -- and uses max(1e-5, 4 x self-spread) per metric.  Where CG converges or stays well
inside the Krylov space the self-spread is far below 1e-5 and the fixed bar is what applies.
"""

import numpy as np
import pytest
import torch
from scipy.linalg import eigvalsh_tridiagonal

import synth
from oracle import cofem, cg as ocg, probes as oprobes, slq
from gpu_common import (DEV, device_model, alpha_dev, log_pi_dev, compare_estep, estep_errors,
                        rel_cols, kappa_hat)
from paper_2310_00420_amd._lib import CMTCS_CG_BREAKDOWN as BREAKDOWN, \
    CMTCS_CG_NONPOS_RITZ as NONPOS_RITZ

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _policy(cfg):
    return ocg.CGPolicy(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters)


def _oracle_columnwise(w, b, alpha, K, pol, seed, it, probes, tasks, precond=None):
    """The oracle with its operator applied one column at a time: the same arithmetic in a
    different FP64 summation order (used only to measure that order's effect)."""
    orig = cofem._cg.cg

    def cg_cols(apply_A, B, policy):
        def ap(V, cols):
            return np.stack([apply_A(V[:, i:i + 1], cols[i:i + 1])[:, 0]
                             for i in range(V.shape[1])], axis=1)
        return orig(ap, B, policy)

    orig_p = cofem._cg.pcg

    def pcg_cols(apply_A, B, policy, m):
        def ap(V, cols):
            return np.stack([apply_A(V[:, i:i + 1], cols[i:i + 1])[:, 0]
                             for i in range(V.shape[1])], axis=1)
        return orig_p(ap, B, policy, m)

    cofem._cg.cg = cg_cols
    cofem._cg.pcg = pcg_cols
    try:
        return cofem.estep(w.phi_list(), b, w.beta, alpha, w.log_pi, K, pol, seed=seed, it=it,
                           probes=probes, t_sel=tasks, precond=precond)
    finally:
        cofem._cg.cg = orig
        cofem._cg.pcg = orig_p


def _run(w, tasks, math="f64", probes=None, seed=1, it=0, alpha=None, K=None, spread=True,
         precond=False):
    cfg = w.cfg
    K = cfg.K if K is None else K
    # the library takes alpha in float32: the oracle gets the same values
    alpha = np.asarray(w.alpha0 if alpha is None else alpha, np.float32).astype(np.float64)
    m = device_model(w, math=math, K=K)
    pr = None if probes is None else torch.tensor(probes.astype(np.int8), device=DEV)
    g = m.estep(alpha_dev(alpha), log_pi_dev(w.log_pi), K, fixed_iters=cfg.fixed_iters,
                tol=cfg.tol, max_iters=cfg.max_iters, seed=seed, em_iter=it, probes=pr,
                stats=True, precond=precond)
    torch.cuda.synchronize()
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    pc = "jacobi" if precond else None
    ref = cofem.estep(w.phi_list(), b, w.beta, alpha, w.log_pi, K, _policy(cfg), seed=seed,
                      it=it, probes=probes, t_sel=tasks, precond=pc)
    err = compare_estep(g, ref, tasks)
    err["kappa_hat"] = kappa_hat(g, tasks)
    # every probe entered the log-determinant average (no non-positive Ritz value)
    assert (g["k_eff"].cpu().numpy() == K).all()
    assert not (g["status"].cpu().numpy() == NONPOS_RITZ).any()
    it_g = g["iters"].cpu().numpy()[np.asarray(tasks)]
    it_o = ref["iters"].reshape(len(tasks), -1)
    err["iters_maxdiff"] = int(np.max(np.abs(it_g - it_o)))
    if spread:
        alt = _oracle_columnwise(w, b, alpha, K, _policy(cfg), seed, it, probes, tasks, pc)
        sp = estep_errors(alt, ref)
        # CG step counts: a column may stop where either FP64 order of the oracle stops (+-1)
        it_a = alt["iters"].reshape(len(tasks), -1)
        err["iters_excess"] = int(np.max(np.abs(it_g - it_o) - np.maximum(1, np.abs(it_a - it_o))))
        print("\noracle self-spread (summation order):",
              {k: float(np.max(v)) for k, v in sp.items()})
    else:
        sp = {k: np.zeros_like(v) for k, v in err["per"].items()}
    err["bar_ratio"] = {k: float(np.max(err["per"][k] / np.maximum(TOL, 4 * sp[k])))
                        for k in sp}
    print("%s math=%s tasks=%s: %s" % (cfg.name, math, list(tasks),
                                       {k: v for k, v in err.items() if k != "per"}))
    m.close()
    return err, g, ref, sp


METRICS = ("mu", "s", "mu_inf", "s_inf", "logdet", "ell")


def _assert(err, spread):
    """Every (t, c) entry within max(1e-5, 4 x the oracle's self-spread of that entry)."""
    for k in METRICS:
        assert err["bar_ratio"][k] <= 1.0, (k, err["bar_ratio"], err[k])
    assert err["argmax_equal"], err


def test_estep_tiny_f64():
    """Plain method, tiny config as specified: fixed 64 CG steps (= D), K = 16, all tasks.
    Bar: max(1e-5, 4 x the oracle's own summation-order spread) -- see the module docstring."""
    w = synth.make("tiny")
    err, g, ref, sp = _run(w, range(w.T))
    _assert(err, sp)
    assert err["iters_maxdiff"] == 0           # fixed mode: every column takes 64 steps


def _ritz_errors(g, ref, tasks, K):
    """Largest relative difference of the device's extreme Ritz values (stats ritz_min/ritz_max)
    from the eigenvalues of the oracle's tridiagonal of Eq. (tridiag) for the same probe."""
    rmin, rmax = g["ritz_min"].cpu().numpy(), g["ritz_max"].cpu().numpy()
    worst = 0.0
    for a, t in enumerate(tasks):
        for c in range(rmin.shape[1]):
            for k in range(K):
                j = c * (K + 1) + 1 + k
                d, e = slq.tridiagonal(ref["gammas"][a][j], ref["xis"][a][j])
                lam = eigvalsh_tridiagonal(d, e) if len(d) > 1 else d
                worst = max(worst, abs(rmin[t, c, k] - lam.min()) / lam.max(),
                            abs(rmax[t, c, k] - lam.max()) / lam.max())
    return worst


def test_estep_tiny_converged_f64():
    """Tiny problem with CG run to convergence (tol 1e-13, at most 10 D steps): the solution is
    unique up to rounding, so the fixed bar applies (the oracle's self-spread here is ~1e-11).
    The extreme Ritz values of every probe's tridiagonal match the oracle's eigenvalues."""
    w = synth.make(synth.Config("tiny-conv", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16,
                                tol=1e-13, max_iters=640))
    err, g, ref, sp = _run(w, range(w.T))
    _assert(err, sp)
    assert max(float(np.max(v)) for v in sp.values()) < 1e-8   # converged: unique up to rounding
    assert (g["status"].cpu().numpy() == 0).all()
    ritz = _ritz_errors(g, ref, range(w.T), w.cfg.K)
    print("ritz values vs oracle eigenvalues: %.2e" % ritz)
    assert ritz < 1e-6


def test_estep_fp32_config_f64_sampled_tasks():
    """Plain FP32 config shape (T=32, C=4, D=1024, N=256, K=32, tol 1e-6, 200 steps): the whole
    batch runs on the device; the oracle checks a sample of tasks from each true cluster."""
    w = synth.make("fp32")
    err, g, ref, sp = _run(w, [0, 9, 18, 31])
    _assert(err, sp)
    assert err["iters_excess"] <= 0


def test_estep_precision_config_f64_sampled_tasks():
    """The measured workload exactly as the benchmark runs it (T=64, C=4, D=4096, N=1024, K=32,
    tol 1e-6, <= 200 steps, FP64, the autotuner's tile shapes): the whole batch of 8448
    right-hand sides on the device; the oracle checks one task from each of two true clusters."""
    w = synth.make("prec")
    err, g, ref, sp = _run(w, [0, 40])
    _assert(err, sp)
    assert err["iters_excess"] <= 0


def test_estep_batch_config_f64_sampled_tasks():
    """Batching configuration: T=256 tasks with N_t ~ U{128..2048} (sum 272,620 rows), D=2048,
    C=8, K=32 -- all 67,584 right-hand sides in one batched solve on the device; the oracle
    checks the two smallest tasks and the median one."""
    w = synth.make("batch")
    ns = np.diff(w.row_off)
    order = np.argsort(ns, kind="stable")
    tasks = sorted([int(order[0]), int(order[1]), int(order[len(order) // 2])])
    err, g, ref, sp = _run(w, tasks)
    _assert(err, sp)
    assert err["iters_excess"] <= 0


@pytest.mark.parametrize("D", [8192, 16384])
def test_estep_largest_d_f64(D):
    """The two widest column shapes of the CG kernels (1024 threads with 8 and 16 elements each)
    up to the largest supported D, with ragged tasks.  beta = 1 and alpha in (1, 2) make the
    systems well conditioned (condition ~ D / N_t), so CG converges to tol 1e-10 and the
    solution is unique up to rounding; at the configurations' beta = 1e4 and a few dozen fixed
    steps the oracle moves by up to 2% with its own summation order and pins nothing."""
    w = synth.make(synth.Config("wide", T=2, C=2, D=D, N=[48, 17], sparsity=8, groups=2, K=3,
                                tol=1e-10, max_iters=400, sigma=1.0))
    err, g, ref, sp = _run(w, range(w.T), alpha=w.alpha0 + 1.0)
    _assert(err, sp)
    assert (g["status"].cpu().numpy() == 0).all()


def test_estep_ragged_edge_f64():
    """Ragged N_t including an empty task, D spanning several tiles with a partial last one,
    C*(K+1) not a multiple of 16, tolerance mode."""
    w = synth.make(synth.Config("ragged", T=6, C=3, D=80, N=[0, 7, 33, 16, 50, 4], sparsity=5,
                                groups=3, K=5, tol=1e-12, max_iters=400))
    assert list(np.diff(w.row_off)) == [0, 7, 33, 16, 50, 4]
    # prior precisions in (1, 2): condition numbers ~1e5, so every solve converges
    err, g, ref, sp = _run(w, range(w.T), alpha=w.alpha0 + 1.0)
    _assert(err, sp)
    assert (g["status"].cpu().numpy() == 0).all()


def test_estep_explicit_probes_f64():
    """Caller-supplied probe buffer (here the generated ones, passed explicitly) gives the same
    result as the generated path."""
    w = synth.make(synth.Config("tiny-conv", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16,
                                tol=1e-13, max_iters=640))
    pr = oprobes.rademacher(7, 3, w.T, w.cfg.C, w.cfg.K, w.cfg.D)
    err1, g1, _, sp = _run(w, range(w.T), probes=pr, seed=7, it=3)
    _assert(err1, sp)
    m = device_model(w)
    g2 = m.estep(alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, tol=1e-13, max_iters=640,
                 seed=7, em_iter=3)
    for k in ("mu", "s", "logdet", "ell", "q"):
        assert torch.equal(g1[k], g2[k]), k


def test_estep_deterministic():
    """Two identical calls give bit-identical outputs (fixed reduction order)."""
    w = synth.make("tiny")
    m = device_model(w)
    a = [m.estep(alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, fixed_iters=64)
         for _ in range(2)]
    for k in a[0]:
        assert torch.equal(a[0][k], a[1][k]), k


def test_responsibilities_sum_to_one():
    w = synth.make("tiny")
    m = device_model(w)
    g = m.estep(alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, fixed_iters=64)
    q = g["q"].cpu().numpy()
    print("\nq", q, "sum-1", q.sum(1) - 1)
    assert np.all(np.abs(q.sum(1) - 1) < 1e-14)


def test_mstep_parity():
    """M-step (Eq. (mstep)) with guards, from identical FP32 mu, s and FP64 q, including a
    non-positive denominator (alpha_max branch) and an empty cluster (alpha kept)."""
    rng = np.random.default_rng(5)
    T, C, D = 7, 3, 96
    mu = rng.standard_normal((T, C, D)).astype(np.float32)
    s = np.abs(rng.standard_normal((T, C, D))).astype(np.float32) * 0.1
    s[:, 0, :5] = -mu[:, 0, :5] ** 2 - 1.0          # den < 0 for c = 0, d < 5
    q = rng.random((T, C)); q[:, 2] = 0.0             # cluster 2 is empty
    q /= q.sum(1, keepdims=True)
    alpha0 = rng.random((C, D)).astype(np.float32) + 0.1
    ref = cofem.mstep(mu, s, q, alpha0.astype(np.float64), alpha_max=1e10)
    w = synth.make(synth.Config("m", T=T, C=C, D=D, N=8, sparsity=3, groups=1, K=1))
    m = device_model(w)
    a = alpha_dev(alpha0)
    m.mstep(torch.tensor(mu, device=DEV), torch.tensor(s, device=DEV),
            torch.tensor(q, device=DEV), a, alpha_max=1e10)
    got = a.cpu().numpy().astype(np.float64)
    ref32 = ref.astype(np.float32).astype(np.float64)
    assert np.all(got[:, :][:2] > 0)
    assert np.max(np.abs(got - ref32) / ref32) <= 2 ** -23
    assert np.all(got[2] == alpha0[2])
    assert np.all(got[0, :5] == np.float32(1e10))


def test_em_iterations_f64():
    """Three EM iterations (E-step + M-step each) on the tiny problem with converged CG: alpha,
    the assignments and the reconstructions track the oracle's trajectory."""
    from paper_2310_00420_amd import fit
    w = synth.make(synth.Config("tiny-conv", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16,
                                tol=1e-13, max_iters=640))
    m = device_model(w)
    out = fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, 3, tol=1e-13,
              max_iters=640)
    ref = cofem.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, w.cfg.K,
                    _policy(w.cfg), 3, seed=1)
    inv_g = 1.0 / out["alpha"].cpu().numpy().astype(np.float64)
    inv_o = 1.0 / ref["alpha"]
    e_alpha = rel_cols(inv_g, inv_o)
    e_mu = rel_cols(out["mu"].cpu().numpy(), ref["mu"])
    print("\nEM x3 tiny: 1/alpha rel %.2e, mu rel %.2e" % (e_alpha, e_mu))
    assert np.array_equal(out["assign"], ref["assign"])
    assert e_alpha <= TOL and e_mu <= TOL


def test_slq_workspace_form_matches_lds_form(monkeypatch):
    """The log-determinant kernel with the tridiagonals in the HBM workspace (the form used past
    4096 CG steps, forced here with CMTCS_SLQ_LDS_BYTES=0) gives bit-identical log-determinants,
    responsibilities and extreme Ritz values to the LDS form, on the same E-step."""
    w = synth.make("fp32", T=8)
    kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=1, em_iter=0, stats=True)
    out = []
    for budget in (None, "0"):
        if budget is None:
            monkeypatch.delenv("CMTCS_SLQ_LDS_BYTES", raising=False)
        else:
            monkeypatch.setenv("CMTCS_SLQ_LDS_BYTES", budget)
        m = device_model(w)
        out.append(m.estep(alpha_dev(w.alpha0), log_pi_dev(w.log_pi), w.cfg.K, **kw))
        torch.cuda.synchronize()
        m.close()
    for k in ("logdet", "ell", "q", "ritz_min", "ritz_max", "iters"):
        assert torch.equal(out[0][k], out[1][k]), k


# ------------------------------------------------------------------------------------------
# Fixed bars where the answer is unique: converged CG on well-conditioned systems.

def _assert_fixed(err):
    for k in METRICS:
        assert err[k] <= TOL, (k, err[k])
    assert err["argmax_equal"], err


def _batch_geometry():
    """The batching configuration's geometry (T=256, N_t ~ U{128..2048}, D=2048, C=8, K=32)
    with beta = 1 and alpha in (1, 2): condition numbers ~10, so CG converges to tol 1e-10 and
    the solutions are unique up to rounding."""
    w = synth.make("batch", sigma=1.0, tol=1e-10, max_iters=400)
    ns = np.diff(w.row_off)
    order = np.argsort(ns, kind="stable")
    tasks = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    return w, tasks


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_estep_batch_geometry_converged(math):
    """All 67,584 right-hand sides of the ragged batching geometry in one solve, FP64 and FP32;
    the oracle checks the smallest, the median and the largest task at the fixed 1e-5 bar, with
    no allowance for the oracle's own spread (it is ~1e-12 here)."""
    w, tasks = _batch_geometry()
    err, g, ref, sp = _run(w, tasks, math=math, alpha=w.alpha0 + 1.0, spread=False)
    print("N_t of the sampled tasks:", [int(n) for n in np.diff(w.row_off)[tasks]])
    _assert_fixed(err)
    assert (g["status"].cpu().numpy() == 0).all()


def test_estep_f32_well_conditioned_fp32_shape():
    """The plain FP32 path at the FP32 configuration's shape (T=32, C=4, D=1024, N=256, K=32)
    with beta = 1 and alpha in (1, 2): every sampled task within the fixed 1e-5 bar."""
    w = synth.make("fp32", sigma=1.0)
    err, g, ref, sp = _run(w, [0, 9, 18, 31], math="f32", alpha=w.alpha0 + 1.0, spread=False)
    _assert_fixed(err)


# ------------------------------------------------------------------------------------------
# The plain FP32 path at the configurations' own conditioning (beta = 1e4, alpha ~ U(0, 1)).
# A rounded operator departs from the FP64 result by ~kappa u (tests/test_precision_emulation.py
# shows this for the arithmetic alone), so FP32 cannot meet 1e-5 there.  Checked here: the
# device's departure is the one FP32 arithmetic itself causes -- within 5x of the CPU model of
# the FP32 form (tests/emulate.py) on the same inputs and probes -- and the 1e-5 bar, which is
# expected to fail (strict xfail).

_F32_CACHE = {}


def _f32_config(name):
    if name in _F32_CACHE:
        return _F32_CACHE[name]
    import emulate
    w = synth.make(name)
    if name == "fp32":
        tasks = [0, 9, 18, 31]
    else:
        ns = np.diff(w.row_off)
        order = np.argsort(ns, kind="stable")
        tasks = sorted([int(order[0]), int(order[1]), int(order[len(order) // 2])])
    err, g, ref, sp = _run(w, tasks, math="f32", spread=False)
    emu = emulate.errors(emulate.estep(w, tasks, w.alpha0, w.cfg.K, emulate.policy_of(w.cfg),
                                       prod="f32", vec="f32"),
                         dict(mu=ref["mu"], s=ref["s"], nu=ref["nu"]))
    print("%s FP32: device mu %.2e s %.2e nu %.2e ell %.2e | CPU model of FP32 mu %.2e s %.2e "
          "nu %.2e | kappa-hat %.2e" % (name, err["mu"], err["s"], err["logdet"], err["ell"],
                                        emu["mu"], emu["s"], emu["nu"], err["kappa_hat"]))
    _F32_CACHE[name] = (err, emu)
    return err, emu


@pytest.mark.parametrize("name", ["fp32", "batch"])
def test_estep_f32_config_departure_is_fp32_rounding(name):
    err, emu = _f32_config(name)
    for k, ke in (("mu", "mu"), ("s", "s"), ("logdet", "nu")):
        assert err[k] <= 5 * emu[ke] + TOL, (k, err[k], emu[ke])
    assert err["argmax_equal"], err


@pytest.mark.xfail(strict=True, reason="FP32 rounding at the configuration's conditioning "
                   "(kappa ~1e8) moves mu by ~1e-1, far above 1e-5; see "
                   "tests/test_precision_emulation.py")
def test_estep_f32_fp32_config_meets_1e5():
    err, emu = _f32_config("fp32")
    _assert_fixed(err)


# ------------------------------------------------------------------------------------------
# The tiny configuration as specified for the plain method: 20 EM iterations of Alg. 2 against
# exact dense EM.  Hadamard probes (K = D = 64 columns of a Sylvester-Hadamard matrix, passed
# explicitly) make the diagonal and log-determinant estimators exact when CG converges, so
# CoFEM's trajectory is dense EM's (Eqs. (estep), (mstep)).

def test_em_trajectory_tiny_hadamard_equals_dense_em():
    from oracle import dense_em
    from paper_2310_00420_amd import fit
    w = synth.make("tiny")
    D, C, n_em = w.cfg.D, w.cfg.C, 20
    H = synth.hadamard(6)
    pr = torch.tensor(np.ascontiguousarray(np.broadcast_to(H[None, None], (w.T, C, D, D)),
                                           dtype=np.int8), device=DEV)
    m = device_model(w, K=D, max_iters=10 * D)
    hist = []

    def keep(it, alpha, out):
        hist.append((alpha.cpu().numpy().astype(np.float64), out["ell"].cpu().numpy(),
                     out["q"].cpu().numpy()))

    out = fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), D, n_em, tol=1e-13,
              max_iters=10 * D, probes_fn=lambda it: pr, callback=keep)
    ref = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, n_em)
    const = cofem.log_norm_const(w.phi_list(), w.y_list(), w.beta)
    worst_a = worst_L = 0.0
    for (a, ell, q), hr in zip(hist, ref["history"]):
        L = cofem.log_likelihood(ell, w.log_pi, const)
        worst_L = max(worst_L, abs(L - hr["L"]) / abs(hr["L"]))
        worst_a = max(worst_a, np.max(np.abs(1 / a - 1 / hr["alpha"])) / np.max(1 / hr["alpha"]))
    print("\n20 EM iterations, Hadamard probes vs dense EM: 1/alpha %.2e, L %.2e"
          % (worst_a, worst_L))
    # the library's M-step returns alpha in float32 (a relative rounding of 6e-8 per iteration,
    # carried through the trajectory), where the oracle keeps FP64: bar 1e-6 on both
    assert worst_a <= 1e-6 and worst_L <= 1e-6
    assert np.array_equal(out["assign"], ref["assign"])
