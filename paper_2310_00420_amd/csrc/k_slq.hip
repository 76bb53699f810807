// Log-determinant by stochastic Lanczos quadrature from the CG coefficients (Sec. 3.2).
//
// For probe k of pair (t, c), the U steps of Alg. 1 on A x = p from x = 0 define the U x U
// symmetric tridiagonal Gamma-bar of Eq. (tridiag):
//     diag_1 = 1/gamma_1,  diag_u = 1/gamma_u + xi_{u-1}/gamma_{u-1},
//     off_{u-1} = sqrt(xi_{u-1})/gamma_{u-1}.
// With Gamma-bar = S^T diag(lambda) S, the quadrature of Eq. (hutch-trace) truncated to U steps
// is  tau = ||p||^2 sum_u S_{u,1}^2 log lambda_u  (the paper's factor D equals ||p||^2 for
// Rademacher probes), and Eq. (logdet-est) averages -tau over the probes.
//
// Only the eigenvalues and the first component of each unit eigenvector are needed (Gauss
// quadrature weights), so the eigensolver is the implicit-shift symmetric QR iteration with
// Wilkinson shifts (Golub & Van Loan, Matrix Computations, Sec. 8.3) that rotates one row
// vector z = e_1^T Q instead of the whole eigenvector matrix: O(U^2) work per probe.
// One thread per probe; its three length-U FP64 arrays live in a workspace laid out
// [u][probe] so that the 64 lanes of a wave touch consecutive addresses.
#include "internal.h"

namespace cmtcs {

// Eigenvalues (left in dg) and first eigenvector components (left in zz, which must enter as
// e_1) of the symmetric tridiagonal with diagonal dg[0..n-1] and off-diagonal of[0..n-2];
// element i of each array is at index i * stride.  Returns 0 on success, 1 if the sweep limit
// was reached.
__host__ __device__ inline int tridiag_eig_first_row(double* dg, double* of, double* zz, int n,
                                                     long stride, int max_sweeps) {
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int sweeps = 0;
  while (hi > 0) {
    const double e_hi = of[(long)(hi - 1) * stride];
    if (fabs(e_hi) <= eps * (fabs(dg[(long)(hi - 1) * stride]) + fabs(dg[(long)hi * stride]))) {
      of[(long)(hi - 1) * stride] = 0.0;
      --hi;
      continue;
    }
    // start of the unreduced block that ends at hi
    int lo = hi - 1;
    while (lo > 0) {
      const double e = of[(long)(lo - 1) * stride];
      if (fabs(e) <= eps * (fabs(dg[(long)(lo - 1) * stride]) + fabs(dg[(long)lo * stride]))) {
        of[(long)(lo - 1) * stride] = 0.0;
        break;
      }
      --lo;
    }
    if (++sweeps > max_sweeps) return 1;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer its last diagonal entry
    const double a = dg[(long)(hi - 1) * stride], bq = of[(long)(hi - 1) * stride];
    const double cq = dg[(long)hi * stride];
    const double delta = 0.5 * (a - cq);
    const double den = delta + copysign(hypot(delta, bq), delta);
    const double mu = cq - bq * bq / den;
    // bulge chase: rotations in planes (k, k+1), k = lo..hi-1
    double x = dg[(long)lo * stride] - mu;
    double y = of[(long)lo * stride];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, y);
      double cs = 1.0, sn = 0.0;
      if (r > 0.0) { cs = x / r; sn = y / r; }
      if (k > lo) of[(long)(k - 1) * stride] = r;
      const double a0 = dg[(long)k * stride], a1 = dg[(long)(k + 1) * stride];
      const double b0 = of[(long)k * stride];
      dg[(long)k * stride] = cs * cs * a0 + 2.0 * cs * sn * b0 + sn * sn * a1;
      dg[(long)(k + 1) * stride] = sn * sn * a0 - 2.0 * cs * sn * b0 + cs * cs * a1;
      const double nb = cs * sn * (a1 - a0) + (cs * cs - sn * sn) * b0;
      of[(long)k * stride] = nb;
      if (k + 1 < hi) {
        const double b1 = of[(long)(k + 1) * stride];
        y = sn * b1;
        of[(long)(k + 1) * stride] = cs * b1;
        x = nb;
      }
      const double z0 = zz[(long)k * stride], z1 = zz[(long)(k + 1) * stride];
      zz[(long)k * stride] = cs * z0 + sn * z1;
      zz[(long)(k + 1) * stride] = -sn * z0 + cs * z1;
    }
  }
  return 0;
}

__global__ __launch_bounds__(64) void k_slq(const double* __restrict__ gam,
                                            const double* __restrict__ xi,
                                            const int* __restrict__ iters, int T, int C, int K,
                                            int Rp, double pnorm2, double* __restrict__ dg,
                                            double* __restrict__ of, double* __restrict__ zz,
                                            double* __restrict__ tau, uint8_t* __restrict__ ok,
                                            double* __restrict__ rmin,
                                            double* __restrict__ rmax) {
  const long P = (long)T * C * K;
  const long p = (long)blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  const int t = (int)(p / ((long)C * K));
  const int c = (int)((p / K) % C);
  const int k = (int)(p % K);
  const long idx = (long)t * Rp + (long)c * (K + 1) + 1 + k;
  const long ncol = (long)T * Rp;
  const int n = iters[idx];
  if (n == 0) {
    tau[p] = 0.0; ok[p] = 0; rmin[p] = NAN; rmax[p] = NAN;
    return;
  }
  double gprev = 1.0, xprev = 0.0;
  for (int u = 0; u < n; ++u) {
    const double g = gam[(long)u * ncol + idx];
    dg[(long)u * P + p] = 1.0 / g + (u > 0 ? xprev / gprev : 0.0);
    if (u + 1 < n) {
      const double x = xi[(long)u * ncol + idx];
      of[(long)u * P + p] = sqrt(x) / g;
      xprev = x;
    }
    zz[(long)u * P + p] = (u == 0) ? 1.0 : 0.0;
    gprev = g;
  }
  const int fail = tridiag_eig_first_row(dg + p, of + p, zz + p, n, P, 30 * n);
  double acc = 0.0, lo = INFINITY, hi = -INFINITY;
  bool pos = true;
  for (int u = 0; u < n; ++u) {
    const double lam = dg[(long)u * P + p];
    const double z = zz[(long)u * P + p];
    lo = fmin(lo, lam);
    hi = fmax(hi, lam);
    if (!(lam > 0.0)) pos = false;
    else acc += z * z * log(lam);
  }
  tau[p] = pnorm2 * acc;
  ok[p] = (pos && !fail) ? 1 : 0;
  rmin[p] = lo;
  rmax[p] = hi;
}

hipError_t launch_slq(const Geometry& g, const CgState& s, int K, double pnorm2, double* dg,
                      double* of, double* zz, double* tau, uint8_t* ok, double* rmin,
                      double* rmax, hipStream_t st) {
  const long P = (long)g.T * g.C * K;
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slq, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, s.gam, s.xi,
                     s.iters, g.T, g.C, K, g.Rp, pnorm2, dg, of, zz, tau, ok, rmin, rmax);
  return hipGetLastError();
}

}  // namespace cmtcs
