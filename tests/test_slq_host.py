"""The SLQ kernel's tridiagonal eigensolver (implicit-shift QR tracking the first row of the
eigenvector matrix), compiled for the host from the same source, against LAPACK's symmetric
tridiagonal eigensolver (scipy.linalg.eigh_tridiagonal).

Checked: eigenvalues; the Gauss quadrature sums sum_i w_i f(lambda_i) for smooth f (the weights
of a repeated eigenvalue are not unique, their sums are); weights summing to 1; and the log
quadrature of Eq. (hutch-trace) on tridiagonals of the form Eq. (tridiag) builds from CG step
sizes.  Cases span sizes 1..220, random, CG-like, split (negligible or zero off-diagonals) and
repeated eigenvalues."""

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


def _cases():
    rng = np.random.default_rng(0)
    cases = []
    for trial in range(240):
        n = int(rng.integers(1, 221))
        kind = trial % 5
        if kind == 0:
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1)
        elif kind == 1:   # Eq. (tridiag) from CG step sizes: positive definite, widely spread
            g = 10 ** rng.uniform(-5, 0, n)
            x = 10 ** rng.uniform(-3, 0.5, n)
            d = 1 / g
            d[1:] += x[:-1] / g[:-1]
            e = np.sqrt(x[:-1]) / g[:-1]
        elif kind == 2:   # negligible off-diagonals: the matrix splits
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1) * 1e-20
        elif kind == 3:   # all eigenvalues clustered in pairs
            d = np.ones(n)
            e = np.ones(n - 1)
        else:             # exact zeros inside: blocks that split in the middle
            d = rng.standard_normal(n)
            e = rng.standard_normal(n - 1)
            e[rng.random(n - 1) < 0.2] = 0.0
        cases.append((kind, d, e))
    return cases


def _run(driver, cases):
    inp = "".join("%d\n%s\n%s\n" % (len(d), " ".join("%.17g" % v for v in d),
                                    " ".join("%.17g" % v for v in e)) for _, d, e in cases)
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    res, pos = [], 0
    for _, d, _ in cases:
        n, fail = map(int, lines[pos].split())
        pos += 1
        v = np.array([[float(x) for x in lines[pos + i].split()] for i in range(n)])
        pos += n
        assert n == len(d)
        res.append((fail, v[:, 0], v[:, 1]))
    return res


def test_eigensolver_matches_lapack(driver):
    cases = _cases()
    worst = dict(eig=0.0, quad=0.0, wsum=0.0, logq=0.0)
    for (kind, d, e), (fail, lam2, w2) in zip(cases, _run(driver, cases)):
        assert fail == 0
        if len(d) > 1:
            lam, S = eigh_tridiagonal(d, e)
            w = S[0] ** 2
        else:
            lam, w = d.copy(), np.ones(1)
        o = np.argsort(lam2)
        lam2, w2 = lam2[o], w2[o]
        sc = np.abs(lam).max()
        worst["eig"] = max(worst["eig"], np.abs(lam2 - lam).max() / sc)
        for f in (lambda v: v, lambda v: v ** 2, lambda v: np.exp(v / sc)):
            a, b = np.sum(w2 * f(lam2)), np.sum(w * f(lam))
            worst["quad"] = max(worst["quad"], abs(a - b) / np.sum(w * np.abs(f(lam))))
        worst["wsum"] = max(worst["wsum"], abs(w2.sum() - 1))
        if kind == 1:
            a, b = np.sum(w2 * np.log(lam2)), np.sum(w * np.log(lam))
            worst["logq"] = max(worst["logq"], abs(a - b) / abs(b))
    print("\n", {k: "%.1e" % v for k, v in worst.items()})
    assert worst["eig"] < 1e-13
    assert worst["quad"] < 1e-10
    assert worst["wsum"] < 1e-13
    assert worst["logq"] < 1e-8
