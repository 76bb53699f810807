"""FP64 CPU oracle for covariance-free EM (CoFEM) on clustered multi-task compressive sensing.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct restatement of the
method of Lin & Ba, "An efficient algorithm for clustered multi-task compressive sensing"
(arXiv 2310.00420), used to check the HIP implementation.  Only the test suite, the smoke check
(``__graft_entry__.smoke``) and the CPU-baseline leg of ``bench.py`` may import it; the product
path (``paper_2310_00420_amd``) never does, and shares no code with it.

Modules
-------
probes    counter-based Rademacher probes (SplitMix64), Alg. 2 "sample probes", Sec. 3.1
cg        conjugate gradient, Alg. 1, with the stopping policy the paper leaves open
slq       Lanczos tridiagonal from CG coefficients and Gauss quadrature, Eqs. (tridiag),
          (hutch-trace), (logdet-est), Sec. 3.2
cofem     CoFEM E-step / M-step / EM driver, Alg. 2 with Eqs. (estep), (mstep), (diag-est),
          (lin-sys); optional learned cluster weights (the mixture-weight M-step, Sec. 2)
dense_em  exact EM with explicit covariance (Eqs. (estep), (mstep)), the baseline CoFEM replaces;
          used only to pin the CoFEM oracle on tiny inputs
adjoint   dense FP64 reference for x = A(alpha, Phi)^-1 b and its gradients (the differentiation
          form; derived from the operator A of Eq. (lin-sys))

Every floating-point computation is FP64.  Pins (tests/test_oracle_*.py) tie each function to
closed forms, library routines, invariants and published generator outputs.  Parity unpinned:
full EM trajectories with random (non-Hadamard) probes are only checked statistically.
"""

from . import probes, cg, slq, cofem, dense_em, adjoint  # noqa: F401
