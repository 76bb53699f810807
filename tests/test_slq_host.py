"""The SLQ kernel's log-determinant quadrature, compiled for the host from the same source,
against LAPACK's symmetric tridiagonal eigensolver (scipy.linalg.eigh_tridiagonal).

The kernel computes e_1^T log(T) e_1 = sum_i w_i log(lambda_i) (w_i the squared first components
of the unit eigenvectors: the Gauss quadrature of Eq. (hutch-trace)) by the trapezoidal rule on
int_0^inf [1/(1+t) - e_1^T (T + t I)^{-1} e_1] dt in s = log t, and lambda_min, lambda_max by
Sturm-count multisection.  Checked here: the Sturm counts against the exact eigenvalue counts;
the extreme eigenvalues; the positive-definiteness decision; and the log quadrature on
tridiagonals of the form Eq. (tridiag) builds from CG step sizes and on shifted random, split
(negligible or zero off-diagonals) and repeated-eigenvalue matrices.  Sizes 1..220."""

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("slq") / "slq_driver")
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "host", "slq_driver.hip"), "-o", exe]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert p.returncode == 0, p.stdout
    return exe


def _eig(d, e):
    if len(d) == 1:
        return d.copy(), np.ones(1)
    lam, S = eigh_tridiagonal(d, e)
    return lam, S[0] ** 2


def _cases():
    rng = np.random.default_rng(0)
    cases = []
    for trial in range(300):
        n = int(rng.integers(1, 221))
        kind = trial % 6
        if kind == 0:     # indefinite random
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1)
        elif kind == 1:   # Eq. (tridiag) from CG step sizes: positive definite, widely spread
            lg = rng.uniform(-6, 0)
            g = 10 ** rng.uniform(lg, rng.uniform(lg, 1), n)
            x = 10 ** rng.uniform(-3, 0.5, n)
            d = 1 / g
            d[1:] += x[:-1] / g[:-1]
            e = np.sqrt(x[:-1]) / g[:-1]
        elif kind == 2:   # negligible off-diagonals: the matrix splits
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1) * 1e-20
        elif kind == 3:   # eigenvalues clustered in pairs
            d = np.ones(n)
            e = np.ones(n - 1)
        elif kind == 4:   # exact zeros inside: blocks that split in the middle
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1)
            e[rng.random(n - 1) < 0.2] = 0.0
        else:             # random, scaled far from 1
            d = rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 6)
            e = rng.standard_normal(n - 1) * np.abs(d).max() * 0.3
        lam, _ = _eig(d, e)
        spd = kind == 1 or rng.random() < 0.6
        if spd and kind != 1:   # shift to positive definite with a chosen condition number
            sc = np.abs(lam).max()
            d = d - lam.min() + sc * 10.0 ** rng.uniform(-6, 0)
            lam, _ = _eig(d, e)
        sc = np.abs(lam).max()
        xs = rng.uniform(lam.min() - 0.1 * sc, lam.max() + 0.1 * sc, 8)
        cases.append((kind, d, e, xs))
    return cases


def _run(driver, cases):
    inp = "".join("%d\n%s\n%s\n%d\n%s\n" % (len(d), " ".join("%.17g" % v for v in d),
                                            " ".join("%.17g" % v for v in e), len(xs),
                                            " ".join("%.17g" % v for v in xs))
                  for _, d, e, xs in cases)
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    res = []
    for i in range(len(cases)):
        f = lines[2 * i].split()
        counts = [int(v) for v in lines[2 * i + 1].split()]
        res.append((int(f[0]), int(f[1]), float(f[2]), float(f[3]), float(f[4]), counts))
    return res


def test_log_quadrature_matches_lapack(driver):
    cases = _cases()
    worst = dict(count=0, lmin=0.0, lmax=0.0, logq=0.0)
    n_pd = 0
    for (kind, d, e, xs), (n, pd, lmin, lmax, logq, counts) in zip(cases, _run(driver, cases)):
        assert n == len(d)
        lam, w = _eig(d, e)
        sc = np.abs(lam).max()
        for x, c in zip(xs, counts):
            if np.abs(lam - x).min() > 1e-9 * sc:
                worst["count"] = max(worst["count"], abs(c - int(np.sum(lam < x))))
        worst["lmin"] = max(worst["lmin"], abs(lmin - lam.min()) / sc)
        worst["lmax"] = max(worst["lmax"], abs(lmax - lam.max()) / sc)
        if abs(lam.min()) > 1e-10 * sc:
            assert pd == int(lam.min() > 0), (kind, n, lam.min())
        if pd:
            n_pd += 1
            ref = np.sum(w * np.log(lam))
            worst["logq"] = max(worst["logq"],
                                abs(logq - ref) / max(abs(ref), np.sum(w * np.abs(np.log(lam)))))
    print("\n", {k: "%.1e" % v for k, v in worst.items()}, "positive definite:", n_pd)
    assert n_pd >= 150
    assert worst["count"] == 0
    assert worst["lmin"] < 1e-13
    assert worst["lmax"] < 1e-13
    assert worst["logq"] < 1e-10


def test_single_row_and_diagonal(driver):
    """n = 1 (log a) and a diagonal matrix (b = 0: the weight sits on the first entry)."""
    cases = [(0, np.array([3.5]), np.zeros(0), np.array([1.0, 4.0])),
             (0, np.array([0.25, 7.0, 2.0]), np.zeros(2), np.array([0.1, 1.0, 3.0, 8.0]))]
    res = _run(driver, cases)
    n, pd, lmin, lmax, logq, counts = res[0]
    assert pd == 1 and lmin == pytest.approx(3.5, rel=1e-15) and lmax == pytest.approx(3.5)
    assert logq == pytest.approx(np.log(3.5), rel=1e-13)
    assert counts == [0, 1]
    n, pd, lmin, lmax, logq, counts = res[1]
    assert pd == 1 and lmin == pytest.approx(0.25, rel=1e-14) and lmax == pytest.approx(7.0)
    assert logq == pytest.approx(np.log(0.25), rel=1e-13)
    assert counts == [0, 1, 2, 3]
