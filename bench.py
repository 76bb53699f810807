"""Benchmark of the CoFEM hot path on one MI355X.

A step is one EM iteration of Alg. 2 over the whole batch: the E-step (batched CG over all
T*C*(K+1) right-hand sides, diagonal and log-determinant estimators, responsibilities) and the
M-step.  Workload: T=64 tasks, C=4 clusters, D=4096, N_t=1024, K=32 probes, CG tolerance 1e-6
with at most 200 steps, synthetic Gaussian sensing data (see synth/).  Inputs are resident in
device memory before timing starts.

Printed (one JSON line): CG right-hand-side iterations per second over the timed EM iterations
(value), the EM iteration time (ms_per_step), the roofline position of the dominant kernel
(timed with HIP events on the library's stream) and the FP64 oracle's rate on a bounded
sample on the host CPU.  The default FP64 run also reports:
  detail.async    the same EM iterations without kernel timing (the library's asynchronous
                  path: every CG step enqueued, no host waits);
  detail.forms    the plain FP32 form and the bf16 / fp16 precision forms on the same workload:
                  speed, and the error of their first E-step against the FP64 one from the same
                  alpha and probes, with whether it meets the form's bar (1e-5 FP32, 1e-3
                  16-bit); a speedup over FP32 is quoted only for a form that meets its bar;
  detail.forms_well_conditioned  the same at beta = 1, alpha in (1, 2), where the bars are met;
  detail.configs  the plain FP32 configuration (T=32, D=1024) and the ragged batching
                  configuration (T=256, D=2048) timed the same way;
  detail.fourier  the paper's own sensing (Sec. 4): partial-Fourier Phi_t with T=64, C=4,
                  D=4096, N=1024 frequencies, K=32, sigma 0.05;
  detail.jacobi   the timed EM iterations again with Jacobi-preconditioned CG.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}     # MI355X dense matrix-core peaks
HBM_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="prec")
    ap.add_argument("--math", default="f64", choices=["f64", "f32", "mixed"])
    ap.add_argument("--phi16", default="bf16", choices=["bf16", "f16"])
    ap.add_argument("--refine-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-tasks", type=int, default=4)
    ap.add_argument("--graph", action="store_true",
                    help="also time the same EM iterations as replays of the whole iteration "
                         "recorded as one HIP graph (reported under detail)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the short FP32 and bf16-precision runs of the same workload that "
                         "the default FP64 run reports under detail.forms")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of timing, compare single-task, multi-task and clustered "
                         "multi-task CS over the support-difference fraction f (T=8 in two "
                         "groups of 4, N=D/4, 5%% sparsity, sigma=0.05, 50 EM iterations, K=15, "
                         "U=50) and print the errors as one JSON line")
    ap.add_argument("--sweep-d", type=int, default=512)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the short runs of the plain-FP32 and batching configurations that "
                         "the default FP64 run reports under detail.configs")
    ap.add_argument("--step-active", metavar="PATH",
                    help="write the per-step active right-hand sides of each task in the timed "
                         "E-steps to PATH (JSON), for --step-table")
    ap.add_argument("--step-table", nargs=2, metavar=("TRACE_CSV", "ACTIVE_JSON"),
                    help="host only: join a rocprofv3 kernel trace (kernel_trace.csv) of a run "
                         "with --step-active with that file and print, per group of CG steps of "
                         "the last E-step, the product launches' durations against the column "
                         "fragments they multiply (markdown)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy 1 GiB device-to-device three times (a plain copy "
                         "kernel of known size, for scaling HBM byte counters)")
    return ap.parse_args()


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def time_form(Cmtcs, torch, w, dev, math, phi16, refine_every, warmup, steps, alpha0=None):
    """EM iterations of the same workload in another arithmetic form, on a handle of its own:
    (ms per EM iteration, CG RHS-iterations per second, host copy of the first E-step's
    outputs -- EM iteration 0 from alpha0)."""
    cfg = w.cfg
    m = Cmtcs(torch.from_numpy(w.Phi).to(dev), w.row_off, torch.from_numpy(w.y).to(dev), w.beta,
              cfg.C, math=math, max_iters=cfg.max_iters, max_K=cfg.K, phi16=phi16)
    alpha = torch.tensor(w.alpha0 if alpha0 is None else alpha0, dtype=torch.float32, device=dev)
    log_pi = torch.tensor(w.log_pi, device=dev)
    kw = dict(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters, seed=1,
              refine_every=refine_every if math == "mixed" else 0)
    iters = []
    first = None
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        out = m.estep(alpha, log_pi, cfg.K, em_iter=it, stats=True, **kw)
        if it == 0:
            first = host(out)
        m.mstep(out["mu"], out["s"], out["q"], alpha)
        if it >= warmup:
            iters.append(out["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rhs = sum(int(i.sum().item()) for i in iters)
    m.close()
    return 1e3 * dt / steps, rhs / dt, first


def form_error(got, ref, bar):
    """Error of one E-step against another from the same alpha and probes: largest relative
    vector-norm error of mu and s over (t, c), relative error of nu-bar and ell, agreement of
    the argmax of q; and whether all four are within `bar` with the same argmax."""
    def cols(a, r):
        a = a.astype(np.float64); r = r.astype(np.float64)
        return float(np.max(np.linalg.norm(a - r, axis=-1) / np.linalg.norm(r, axis=-1)))
    e = {"mu": cols(got["mu"], ref["mu"]), "s": cols(got["s"], ref["s"]),
         "nu": float(np.max(np.abs(got["logdet"] - ref["logdet"]) / np.abs(ref["logdet"]))),
         "ell": float(np.max(np.abs(got["ell"] - ref["ell"])
                             / np.maximum(np.abs(ref["ell"]), np.abs(ref["logdet"])))),
         "argmax_agree": float(np.mean(got["q"].argmax(1) == ref["q"].argmax(1)))}
    e = {k: (round(v, 6) if k == "argmax_agree" else float("%.3g" % v)) for k, v in e.items()}
    e["bar"] = bar
    e["meets_bar"] = bool(all(e[k] <= bar for k in ("mu", "s", "nu", "ell"))
                          and e["argmax_agree"] == 1.0)
    return e


def forms_block(Cmtcs, torch, w, dev, refine_every, ref_first, f64_ms, alpha0=None):
    """FP32 and the two precision forms against the FP64 E-step `ref_first` (same alpha, same
    probes); a form's speedup over FP32 is given only when both meet their bars."""
    res = {"f64": {"ms_per_step": round(f64_ms, 2)}}
    for name, math, kind, bar in (("f32", "f32", "bf16", 1e-5), ("mixed_bf16", "mixed", "bf16", 1e-3),
                                  ("mixed_f16", "mixed", "f16", 1e-3)):
        ms, v, first = time_form(Cmtcs, torch, w, dev, math, kind, refine_every, 1, 2, alpha0)
        res[name] = {"ms_per_step": round(ms, 2), "value": v,
                     "error_vs_f64": form_error(first, ref_first, bar)}
        if math == "mixed":
            res[name]["refine_every"] = refine_every
    for name in ("mixed_bf16", "mixed_f16"):
        if res[name]["error_vs_f64"]["meets_bar"] and res["f32"]["error_vs_f64"]["meets_bar"]:
            res[name]["speedup_over_f32"] = round(res["f32"]["ms_per_step"]
                                                  / res[name]["ms_per_step"], 3)
    return res


def measured_traffic(kernel, workload, math):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter record
    (profiles/traffic.json), or None if there is none for this workload or the kernel's source
    has changed since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if rec["workload"] != workload or rec["math"] != math:
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]


def cpu_baseline(w, ntasks):
    """The FP64 oracle on a bounded sample: `ntasks` tasks (spread over the true clusters), one
    full E-step with the workload's CG policy."""
    from oracle import cofem, cg as ocg
    blas = "unknown BLAS"
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        if info:
            blas = "%s %s" % (info[0].get("internal_api", "?"), info[0].get("version", "?"))
    except Exception:
        threads = os.cpu_count()
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cfg = w.cfg
    tasks = [int(v) for v in np.linspace(0, cfg.T - 1, ntasks).round()]
    pol = ocg.CGPolicy(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters)
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs([Phi[t] for t in tasks], [y[t] for t in tasks], w.beta)
    b_full = [None] * cfg.T
    for i, t in enumerate(tasks):
        b_full[t] = b[i]
    t0 = time.perf_counter()
    ref = cofem.estep(Phi, b_full, w.beta, w.alpha0, w.log_pi, cfg.K, pol, seed=1, it=0,
                      t_sel=tasks)
    dt = time.perf_counter() - t0
    rhs_iters = int(ref["iters"].sum())
    return {"value": rhs_iters / dt, "unit": "RHS-iters/s", "cores": int(threads),
            "kind": "oracle",
            "cpu": cpu, "blas": blas,
            "sample": "tasks %s of the workload, one E-step (K=%d, tol %g, <=%d CG steps), "
                      "%d RHS-iterations in %.1f s; FP64 numpy on %s, %d threads"
                      % (tasks, cfg.K, cfg.tol, cfg.max_iters, rhs_iters, dt, blas, threads)}


def run_sweep(a):
    import torch
    import synth
    from paper_2310_00420_amd.experiments import compare_methods

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    D = a.sweep_d
    rows = []
    for f in (0.0, 0.25, 0.5, 0.75, 1.0):
        w = synth.make(synth.Config("support-sweep", T=8, C=2, D=D, N=D // 4,
                                    sparsity=max(1, round(0.05 * D)), groups=2, sigma=0.05,
                                    support_diff=f))
        r = compare_methods(torch.from_numpy(w.Phi).to(dev), w.row_off,
                            torch.from_numpy(w.y).to(dev), w.z, w.beta, C=2)
        def found(a):
            return bool(len(set(a[:4])) == 1 and len(set(a[4:])) == 1 and a[0] != a[4])
        rows.append(dict(f=f, single=r["single"], multi=r["multi"], clustered=r["clustered"],
                         clusters_found=found(r["assign"]),
                         clustered_common_probes=r["clustered_common"],
                         clusters_found_common_probes=found(r["assign_common"]),
                         seconds={k: round(v, 3) for k, v in r["seconds"].items()}))
        print("f=%.2f single %.4f multi %.4f clustered %.4f (common probes %.4f)"
              % (f, r["single"], r["multi"], r["clustered"], r["clustered_common"]),
              file=sys.stderr, flush=True)
    print(json.dumps(dict(experiment="support-difference sweep", D=D, N=D // 4, T=8,
                          data="synthetic Gaussian Phi", rows=rows)), flush=True)


def dense_em_iteration(torch, phi, row_off, y, beta, alpha, log_pi, budget=64 << 30):
    """One iteration of standard EM (Eqs. (estep), (mstep)), the comparison method that CoFEM
    replaces, on the same GPU in FP64 through torch.linalg: per task and cluster a Cholesky
    factorisation L of A = beta Phi_t^T Phi_t + diag(alpha_c), mu = A^-1 b_t, the diagonal of
    Sigma = A^-1 = L^-T L^-1 as column sums of (L^-1)^2, log det Sigma = -2 sum log diag L, ell,
    q and the M-step.  A baseline for timing (not part of the library).  phi [sum N_t][D] and y
    float32 on the device; alpha [C][D], log_pi [C] float64 on the device; tasks are processed
    in groups sized to `budget` bytes of factor storage.

    Not called by any timing run: over 256 matrices of order 1024 (T = 64, C = 4) the batched
    factorisation and solves faulted the GPU inside torch.linalg, with no cause established."""
    f64 = torch.float64
    dev = phi.device
    T = len(row_off) - 1
    C, D = alpha.shape
    tb = int(max(1, min(T, budget // (4 * C * D * D * 8))))
    mu = torch.empty(T, C, D, dtype=f64, device=dev)
    var = torch.empty_like(mu)
    logdet = torch.empty(T, C, dtype=f64, device=dev)
    ell = torch.empty_like(logdet)
    sla = torch.log(alpha).sum(dim=1)
    for t0 in range(0, T, tb):
        ts = list(range(t0, min(T, t0 + tb)))
        P = [phi[int(row_off[t]):int(row_off[t + 1])].double() for t in ts]
        yv = [y[int(row_off[t]):int(row_off[t + 1])].double() for t in ts]
        G = torch.stack([beta * (p.T.contiguous() @ p) for p in P])
        b = torch.stack([beta * (p.T.contiguous() @ v) for p, v in zip(P, yv)])
        A = G[:, None] + torch.diag_embed(alpha)[None]
        del G
        L = torch.linalg.cholesky(A)
        del A
        m = torch.cholesky_solve(b[:, None, :, None].expand(-1, C, -1, -1).contiguous(), L)[..., 0]
        eye = torch.eye(D, dtype=f64, device=dev).expand(len(ts), C, D, D)
        Li = torch.linalg.solve_triangular(L, eye, upper=False)
        v = (Li * Li).sum(dim=-2)
        del Li
        ld = -2.0 * torch.log(torch.diagonal(L, dim1=-2, dim2=-1)).sum(dim=-1)
        del L
        mu[t0:t0 + len(ts)] = m
        var[t0:t0 + len(ts)] = v
        logdet[t0:t0 + len(ts)] = ld
        ell[t0:t0 + len(ts)] = ld + sla[None] + (b[:, None, :] * m).sum(dim=-1)
    q = torch.softmax(0.5 * ell + log_pi[None], dim=1)
    den = (q[:, :, None] * (mu * mu + var)).sum(dim=0)
    return dict(mu=mu, var=var, logdet=logdet, ell=ell, q=q, alpha=q.sum(dim=0)[:, None] / den)


def roofline(m, w, math, config, prof, iters):
    """Roofline position of the dominant product over the profiled EM iterations (HIP-event
    kernel time on the library's stream, algorithmic work of the RHS-iterations executed)."""
    cfg = w.cfg
    ns = np.diff(w.row_off).astype(np.float64)
    name = max(("phi_v", "phit_w"), key=lambda k: prof[k][0])
    tot_ms, launches = prof[name]
    if math == "mixed":
        # HBM-bound: algorithmic bytes = the 16-bit Phi stream plus one pass over the vectors,
        # for every step each task is still active (task-steps = its longest column)
        R = cfg.C * (cfg.K + 1)
        task_steps = sum(i.max(dim=1).values.double().cpu().numpy() for i in iters)
        if name == "phi_v":    # Phi16 N D, V16 R D, W16 R N (2-byte elements)
            per_task = 2.0 * (ns * cfg.D + R * cfg.D + R * ns)
        else:                  # PhiT16 D N, W16 R N, V and A V in FP32: 8 R D
            per_task = 2.0 * (ns * cfg.D + R * ns) + 8.0 * R * cfg.D
        nbytes = float((task_steps * per_task).sum())
        achieved = nbytes / (tot_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_GBPS, 4), "traffic": None,
                "kernel": name + "16", "avg_launch_us": round(1e3 * tot_ms / max(launches, 1), 2),
                "bytes_per_launch": nbytes / max(launches, 1)}
    # algorithmic flops = 2 N_t D per RHS-iteration per product (rows weight ragged tasks)
    row_iters = float(sum((i.double().sum(dim=1).cpu().numpy() * ns).sum() for i in iters))
    flops = 2.0 * cfg.D * row_iters
    achieved = flops / (tot_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[math]
    trows = m.tiles()[0 if name == "phi_v" else 1]
    vt = "double" if math == "f64" else "float"
    kname = "k_%s%s<%s, %d>" % (name, "_lds" if trows < 0 else "", vt, abs(trows) // 16)
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(kname, config, math),
            "kernel": kname, "avg_launch_us": round(1e3 * tot_ms / max(launches, 1), 2),
            "flop_per_launch": flops / max(launches, 1)}


def fragment_work(nact, R, group=144):
    """Column fragments (16 columns each) the CG loop's FP64 LDS-staged products multiply for a
    task with `nact` active of R right-hand sides: active columns are compacted into the
    leading fragments of each 144-column group, and a last fragment with at most four active
    columns costs a quarter (4x4x4 products)."""
    work = 0.0
    for g0 in range(0, R, group):
        n = min(max(nact - g0, 0), group)
        if n == 0:
            break
        frags = -(-n // 16)
        work += frags - 0.75 if n - 16 * (frags - 1) <= 4 else frags
    return work


def step_table(trace_csv, active_json):
    """Durations of the product launches of the last E-step in a kernel trace against the
    fragments they multiply (steps grouped by that work, fastest first)."""
    import csv
    act = json.load(open(active_json))
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"].replace("void ", "", 1) for r in rows]
    last_init = max(i for i, n in enumerate(names) if "k_cg_init" in n)
    per = {}
    for r, n in zip(rows[last_init:], names[last_init:]):
        for key in ("k_phi_v", "k_phit_w"):
            if n.startswith("cmtcs::" + key + "_lds<") or n.startswith("cmtcs::" + key + "<"):
                per.setdefault(key, []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    steps = act["active"][-1]            # [step][task] of the last E-step
    R = act["R"]
    work = [sum(fragment_work(n, R) for n in s) for s in steps]
    cols = [sum(s) for s in steps]
    nst = min(len(work), *(len(v) for v in per.values()))
    order = sorted(range(nst), key=lambda u: work[u])
    nb = 8
    out = ["| steps | active columns (mean) | fragments multiplied (mean, of %d) | forward us "
           "(mean) | adjoint us (mean) | adjoint us per 1000 fragments |"
           % (act["T"] * -(-R // 16)), "|---|---|---|---|---|---|"]
    for b in range(nb):
        idx = order[b * nst // nb:(b + 1) * nst // nb]
        if not idx:
            continue
        f = np.mean([per["k_phi_v"][u] for u in idx])
        g = np.mean([per["k_phit_w"][u] for u in idx])
        wk = np.mean([work[u] for u in idx])
        out.append("| %d | %.0f | %.2f | %.1f | %.1f | %.1f |"
                   % (len(idx), np.mean([cols[u] for u in idx]), wk, f, g,
                      1e3 * g / max(wk, 1e-9)))
    return "\n".join(out)


def run_workload(torch, Cmtcs, w, dev, config, math, phi16, refine_every, warmup, steps,
                 unprofiled=False, alpha0=None, precond=False):
    """Times `steps` EM iterations (E-step + M-step, K probes, the workload's CG policy) after
    `warmup` untimed ones, with HIP-event kernel timing on the library's stream; optionally the
    same iterations again without kernel timing.  Returns the measurements and the host copy of
    the first E-step (EM iteration 0 from alpha^0)."""
    cfg = w.cfg
    m = Cmtcs(torch.from_numpy(w.Phi).to(dev), w.row_off, torch.from_numpy(w.y).to(dev), w.beta,
              cfg.C, math=math, max_iters=cfg.max_iters, max_K=cfg.K, phi16=phi16)
    a0 = w.alpha0 if alpha0 is None else alpha0
    alpha = torch.tensor(a0, dtype=torch.float32, device=dev)
    log_pi = torch.tensor(w.log_pi, device=dev)
    kw = dict(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters, seed=1,
              refine_every=refine_every if math == "mixed" else 0, precond=precond)
    first = None

    def em_iteration(it):
        out = m.estep(alpha, log_pi, cfg.K, em_iter=it, stats=True, **kw)
        m.mstep(out["mu"], out["s"], out["q"], alpha)
        return out

    for it in range(warmup):
        out = em_iteration(it)
        if it == 0:
            first = host(out)
    torch.cuda.synchronize()
    m.profile(True)
    iters = []
    t0 = time.perf_counter()
    for it in range(warmup, warmup + steps):
        out = em_iteration(it)
        iters.append(out["iters"])
        if first is None:   # no warm-up: the first timed E-step is EM iteration 0
            first = host(out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = m.profile(False)
    rhs_iters = int(sum(int(i.sum().item()) for i in iters))
    res = {"value": rhs_iters / dt, "ms_per_step": 1e3 * dt / steps,
           "roofline": roofline(m, w, math, config, prof, iters),
           "rhs_iters_per_em_iter": rhs_iters / steps,
           "max_cg_steps": int(max(int(i.max().item()) for i in iters)),
           "tile_rows": m.tiles(),
           "kernel_ms_per_em_iter": {k: round(v[0] / steps, 3) for k, v in prof.items()},
           "launches_per_em_iter": {k: v[1] / steps for k, v in prof.items()}}
    if unprofiled:
        # the same EM iterations from the same alpha^0, without kernel timing: every CG step is
        # enqueued at once and the host never waits inside an E-step
        alpha.copy_(torch.tensor(a0, dtype=torch.float32, device=dev))
        for it in range(warmup):
            em_iteration(it)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(warmup, warmup + steps):
            out2 = em_iteration(it)
        torch.cuda.synchronize()
        adt = time.perf_counter() - t0
        res["async"] = {"ms_per_step": 1e3 * adt / steps, "value": rhs_iters / adt,
                        "same_q_as_profiled": bool(torch.equal(out2["q"], out["q"]))}
    res["_first"] = first
    res["_model"] = (m, alpha, log_pi)
    res["_iters"] = iters
    return res


FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak


def run_fourier_workload(torch, Cmtcs, name, dev, warmup, steps):
    """EM iterations on a partial-Fourier workload (Sec. 4 sensing): the whole CG solve of two
    columns per workgroup in one kernel.  Roofline: FP64 arithmetic of the transforms, counted
    as 5 N log2 N per complex FFT of N = D points (two per step of a column pair, i.e. one per
    RHS-iteration), against the FP64 vector peak."""
    import synth
    w = synth.make_fourier(name)
    cfg = w.cfg
    m = Cmtcs.partial_fourier(torch.tensor(w.freq, device=dev), w.row_off,
                              torch.tensor(w.yc, device=dev), cfg.D, w.beta, cfg.C,
                              max_iters=cfg.max_iters, max_K=cfg.K)
    alpha = torch.tensor(w.alpha0, dtype=torch.float32, device=dev)
    log_pi = torch.tensor(w.log_pi, device=dev)
    kw = dict(tol=cfg.tol, max_iters=cfg.max_iters, seed=1)
    for it in range(warmup):
        out = m.estep(alpha, log_pi, cfg.K, em_iter=it, **kw)
        m.mstep(out["mu"], out["s"], out["q"], alpha)
    torch.cuda.synchronize()
    m.profile(True)
    iters = []
    t0 = time.perf_counter()
    for it in range(warmup, warmup + steps):
        out = m.estep(alpha, log_pi, cfg.K, em_iter=it, stats=True, **kw)
        m.mstep(out["mu"], out["s"], out["q"], alpha)
        iters.append(out["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = m.profile(False)
    m.close()
    rhs = int(sum(int(i.sum().item()) for i in iters))
    ms, launches = prof["cg_update"]
    N = cfg.D
    flops = 5.0 * N * np.log2(N) * rhs
    achieved = flops / (ms * 1e-3) / 1e12
    return {"workload": "partial-Fourier CoFEM EM iteration, T=%d C=%d D=%d N=%d frequencies "
                        "(2N real measurements), K=%d, sigma %g, CG tol %g, <=%d steps"
                        % (cfg.T, cfg.C, cfg.D, cfg.N, cfg.K, cfg.sigma, cfg.tol, cfg.max_iters),
            "math": "f64", "value": rhs / dt, "unit": "RHS-iters/s", "ms_per_step": 1e3 * dt / steps,
            "rhs_iters_per_em_iter": rhs / steps,
            "max_cg_steps": int(max(int(i.max().item()) for i in iters)),
            "solve_kernel_ms_per_em_iter": round(ms / steps, 3),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                         "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / FP64_VECTOR_TFLOPS, 4), "traffic": None,
                         "kernel": "k_fourier_cg<%d>" % int(np.log2(N)),
                         "avg_launch_us": round(1e3 * ms / max(launches, 1), 2),
                         "flop_per_launch": flops / max(launches, 1)}}


def workload_name(cfg):
    return ("CoFEM EM iteration (E-step + M-step), T=%d C=%d D=%d N=%s K=%d, CG tol %g, "
            "<=%d steps" % (cfg.T, cfg.C, cfg.D, cfg.N, cfg.K, cfg.tol, cfg.max_iters))


def main():
    a = parse()
    if a.sweep:
        run_sweep(a)
        return
    if a.step_table:
        print(step_table(*a.step_table))
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (tasks would shard "
              "across GPUs with one all-reduce of the M-step sums per EM iteration; not built). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2310_00420_amd import Cmtcs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.config.startswith("fourier"):
        # the partial-Fourier workload alone (for profiling its solve kernel)
        r = run_fourier_workload(torch, Cmtcs, a.config, dev, a.warmup, a.steps)
        print(json.dumps(r))
        return
    w = synth.make(a.config)
    cfg = w.cfg
    rows = int(w.row_off[-1])
    main_run = a.math == "f64" and a.config == "prec"
    r = run_workload(torch, Cmtcs, w, dev, a.config, a.math, a.phi16, a.refine_every, a.warmup,
                     a.steps, unprofiled=main_run and not a.no_forms)
    m, alpha, log_pi = r.pop("_model")
    first = r.pop("_first")
    iters = r.pop("_iters")
    if a.step_active:
        # active right-hand sides of task t at CG step u: columns that took more than u steps
        R = cfg.C * (cfg.K + 1)
        steps_max = cfg.fixed_iters if cfg.fixed_iters > 0 else cfg.max_iters
        act = []
        for it in iters:
            n = it.cpu().numpy()
            act.append([[int((n[t] > u).sum()) for t in range(cfg.T)] for u in range(steps_max)])
        json.dump({"T": cfg.T, "R": R, "active": act}, open(a.step_active, "w"))
    res = {
        "metric": "CG RHS-iters/sec + EM iter time, D=4096 T=64 C=4 K=32; MFMA/HBM roofline %",
        "value": r["value"], "unit": "RHS-iters/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": a.math if a.math != "mixed" else a.phi16 + "+f32",
        "data": "synthetic: Phi_t iid N(0,1/N) stored fp32, %d true clusters with %d-sparse "
                "shared supports, sigma %g, seeds data %d / init %d / probes 1"
                % (cfg.groups, cfg.sparsity, cfg.sigma, synth.DATA_SEED, synth.INIT_SEED),
        "config": {"workload": workload_name(cfg),
                   "T": cfg.T, "C": cfg.C, "D": cfg.D, "N": cfg.N, "rows": rows, "K": cfg.K,
                   "math": a.math if a.math != "mixed" else
                   "mixed(%s, true residual every %d)" % (a.phi16, a.refine_every)},
        "roofline": r["roofline"],
        "detail": {k: r[k] for k in ("rhs_iters_per_em_iter", "max_cg_steps", "tile_rows",
                                     "kernel_ms_per_em_iter", "launches_per_em_iter")},
    }
    if "async" in r:
        res["detail"]["async"] = r["async"]
    if a.graph and a.math != "mixed":
        # the same EM iterations, each one replay of the recorded iteration (cmtcs_em_iter):
        # bit-identical results, so the same RHS-iteration count
        alpha.copy_(torch.tensor(w.alpha0, dtype=torch.float32, device=dev))
        gkw = dict(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters, seed=1,
                   graph=True)
        gout = None
        for it in range(a.warmup):
            gout = m.em_iter(alpha, log_pi, cfg.K, out=gout, em_iter=it, **gkw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(a.warmup, a.warmup + a.steps):
            gout = m.em_iter(alpha, log_pi, cfg.K, out=gout, em_iter=it, **gkw)
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        res["detail"]["graph"] = {"ms_per_step": 1e3 * gdt / a.steps,
                                  "value": r["rhs_iters_per_em_iter"] * a.steps / gdt}
    m.close()
    if main_run and not a.no_forms:
        res["detail"]["forms"] = forms_block(Cmtcs, torch, w, dev, a.refine_every, first,
                                             r["ms_per_step"])
        print("forms done", file=sys.stderr, flush=True)
        # the same shape with beta = 1 and alpha in (1, 2), where every form can meet its bar
        wc = synth.make(a.config, sigma=1.0)
        rc = run_workload(torch, Cmtcs, wc, dev, a.config, "f64", a.phi16, a.refine_every, 1, 2,
                          alpha0=wc.alpha0 + 1.0)
        rc.pop("_model")[0].close()
        res["detail"]["forms_well_conditioned"] = {
            "workload": "as above with beta = 1, alpha^0 + 1",
            **forms_block(Cmtcs, torch, wc, dev, a.refine_every, rc.pop("_first"),
                          rc["ms_per_step"], alpha0=wc.alpha0 + 1.0)}
        print("well-conditioned forms done", file=sys.stderr, flush=True)
    if main_run and not a.no_configs:
        # the same EM iterations with Jacobi-preconditioned CG (not in the paper)
        rp = run_workload(torch, Cmtcs, w, dev, a.config, "f64", a.phi16, a.refine_every,
                          a.warmup, a.steps, precond=True)
        rp.pop("_model")[0].close()
        rp.pop("_first")
        res["detail"]["jacobi"] = {k: rp[k] for k in ("value", "ms_per_step",
                                                       "rhs_iters_per_em_iter", "max_cg_steps",
                                                       "kernel_ms_per_em_iter")}
        print("jacobi done", file=sys.stderr, flush=True)
        res["detail"]["fourier"] = run_fourier_workload(torch, Cmtcs, "fourier", dev, 1, 2)
        print("fourier done", file=sys.stderr, flush=True)
        configs = {}
        for name, math in (("fp32", "f32"), ("batch", "f32"), ("batch", "f64")):
            wk = synth.make(name)
            rk = run_workload(torch, Cmtcs, wk, dev, name, math, a.phi16, a.refine_every, 1, 2)
            rk.pop("_model")[0].close()
            rk.pop("_first")
            rk.pop("_iters")
            configs["%s_%s" % (name, math)] = {"workload": workload_name(wk.cfg), "math": math,
                                               **rk}
            print("config %s %s done" % (name, math), file=sys.stderr, flush=True)
        res["detail"]["configs"] = configs
    if a.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["detail"]["copy_calibration_bytes"] = 4 << 28
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, a.cpu_tasks)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
