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
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace cmtcs {

// Eigenvalues (left in dg) and first eigenvector components (left in zz, which must enter as
// e_1) of the symmetric tridiagonal with diagonal dg[0..n-1] and off-diagonal of[0..n-2];
// element i of each array is at index i * stride (index type I: int for on-chip arrays).
// Returns 0 on success, 1 if the sweep limit was reached.
// Within a sweep, the entries a rotation has just updated at position k+1 are exactly the ones
// the next rotation reads, so they are carried in registers: each rotation loads only the
// untouched entries at k+1 (and k+2 for the bulge) and stores its finished entries at k.
// Reciprocal square root of r2 > 0 for the Givens rotations.  On the device: the hardware
// estimate refined by two Newton steps (y <- y (3 - r2 y^2) / 2, each roughly squaring the
// relative error), accurate to a few ulp, which is all a rotation needs (cs^2 + sn^2 = 1).
struct RsqDevice {
  __device__ double operator()(double r2) const {
    double y = __builtin_amdgcn_rsq(r2);
    y = y * (1.5 - 0.5 * r2 * y * y);
    y = y * (1.5 - 0.5 * r2 * y * y);
    return y;
  }
};
// The same on the host (used by host-side checks of this routine).
struct RsqHost {
  __host__ double operator()(double r2) const { return 1.0 / std::sqrt(r2); }
};

template <typename I, typename Rsq>
__host__ __device__ inline int tridiag_eig_first_row(double* dg, double* of, double* zz, int n,
                                                     I stride, int max_sweeps, Rsq rsq) {
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int sweeps = 0;
  while (hi > 0) {
    const double e_hi = of[(I)(hi - 1) * stride];
    if (fabs(e_hi) <= eps * (fabs(dg[(I)(hi - 1) * stride]) + fabs(dg[(I)hi * stride]))) {
      of[(I)(hi - 1) * stride] = 0.0;
      --hi;
      continue;
    }
    // start of the unreduced block that ends at hi
    int lo = hi - 1;
    while (lo > 0) {
      const double e = of[(I)(lo - 1) * stride];
      if (fabs(e) <= eps * (fabs(dg[(I)(lo - 1) * stride]) + fabs(dg[(I)lo * stride]))) {
        of[(I)(lo - 1) * stride] = 0.0;
        break;
      }
      --lo;
    }
    if (++sweeps > max_sweeps) return 1;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer its last diagonal entry
    const double a = dg[(I)(hi - 1) * stride], bq = of[(I)(hi - 1) * stride];
    const double cq = dg[(I)hi * stride];
    const double delta = 0.5 * (a - cq);
    const double den = delta + copysign(hypot(delta, bq), delta);
    const double mu = cq - bq * bq / den;
    // bulge chase: rotations in planes (k, k+1), k = lo..hi-1
    double a0 = dg[(I)lo * stride], b0 = of[(I)lo * stride], z0 = zz[(I)lo * stride];
    double x = a0 - mu;
    double y = b0;
    for (int k = lo; k < hi; ++k) {
      const double a1 = dg[(I)(k + 1) * stride];
      const double z1 = zz[(I)(k + 1) * stride];
      const double b1 = (k + 1 < hi) ? of[(I)(k + 1) * stride] : 0.0;
      // Givens rotation zeroing y against x.  The entries are eigenvalue-sized (CG step
      // sizes of a positive definite system), far from FP64 overflow, so r needs no scaling;
      // one reciprocal square root keeps the dependent chain of a step short.
      const double r2 = x * x + y * y;
      double cs = 1.0, sn = 0.0, r = 0.0;
      if (r2 > 0.0) {
        const double inv = rsq(r2);
        r = r2 * inv;
        cs = x * inv;
        sn = y * inv;
      }
      if (k > lo) of[(I)(k - 1) * stride] = r;
      const double na0 = cs * cs * a0 + 2.0 * cs * sn * b0 + sn * sn * a1;
      const double na1 = sn * sn * a0 - 2.0 * cs * sn * b0 + cs * cs * a1;
      const double nb = cs * sn * (a1 - a0) + (cs * cs - sn * sn) * b0;
      dg[(I)k * stride] = na0;
      of[(I)k * stride] = nb;
      zz[(I)k * stride] = cs * z0 + sn * z1;
      z0 = -sn * z0 + cs * z1;
      a0 = na1;
      if (k + 1 < hi) {
        y = sn * b1;      // bulge at (k+2, k)
        b0 = cs * b1;     // off-diagonal (k+1, k+2) after this rotation
        x = nb;
      }
    }
    dg[(I)hi * stride] = a0;
    zz[(I)hi * stride] = z0;
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
  const int fail = tridiag_eig_first_row<long>(dg + p, of + p, zz + p, n, P, 30 * n,
                                               RsqDevice());
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

// The same computation with each probe's three arrays in LDS: PB probes per block (one
// thread each), arrays laid out [u][probe] in dynamic shared memory of 3 * PB * Um doubles.
// Keeping the O(U) working set of a probe on chip removes the global-memory round trips of
// the QR sweeps, which otherwise dominate this kernel.
__global__ __launch_bounds__(64) void k_slq_lds(const double* __restrict__ gam,
                                                const double* __restrict__ xi,
                                                const int* __restrict__ iters, int T, int C,
                                                int K, int Rp, double pnorm2,
                                                double* __restrict__ tau,
                                                uint8_t* __restrict__ ok,
                                                double* __restrict__ rmin,
                                                double* __restrict__ rmax, int PB, int Um) {
  extern __shared__ double sm[];
  const int lp = threadIdx.x;
  if (lp >= PB) return;
  const long P = (long)T * C * K;
  const long p = (long)blockIdx.x * PB + lp;
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
  double* dg = sm + lp;
  double* of = sm + (long)PB * Um + lp;
  double* zz = sm + 2L * PB * Um + lp;
  double gprev = 1.0, xprev = 0.0;
  for (int u = 0; u < n; ++u) {
    const double g = gam[(long)u * ncol + idx];
    dg[(long)u * PB] = 1.0 / g + (u > 0 ? xprev / gprev : 0.0);
    if (u + 1 < n) {
      const double x = xi[(long)u * ncol + idx];
      of[(long)u * PB] = sqrt(x) / g;
      xprev = x;
    }
    zz[(long)u * PB] = (u == 0) ? 1.0 : 0.0;
    gprev = g;
  }
  const int fail = tridiag_eig_first_row<int>(dg, of, zz, n, PB, 30 * n, RsqDevice());
  double acc = 0.0, lo = INFINITY, hi = -INFINITY;
  bool pos = true;
  for (int u = 0; u < n; ++u) {
    const double lam = dg[(long)u * PB];
    const double z = zz[(long)u * PB];
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

hipError_t launch_slq(const Geometry& g, const CgState& s, int K, int steps, double pnorm2,
                      double* dg, double* of, double* zz, double* tau, uint8_t* ok, double* rmin,
                      double* rmax, hipStream_t st) {
  const long P = (long)g.T * g.C * K;
  if (P == 0) return hipSuccess;
  // 16 KB of LDS per block: a few probes per block and many blocks per CU, so that every SIMD
  // has several waves whose sequential QR chains hide each other's latency
  // With few probes, LDS-resident tridiagonals in small blocks spread the probes over every
  // SIMD; with many (more than fit on chip in one round), one probe per lane in full waves keeps
  // more probes in flight at once and the global-memory layout wins.
  constexpr long kLdsBytes = 16 * 1024;
  constexpr long kLdsMaxProbes = 16384;
  const long Um = steps > 0 ? steps : 1;
  const long PB = std::min<long>(64, kLdsBytes / (24 * Um));
  if (PB >= 1 && P <= kLdsMaxProbes) {
    hipLaunchKernelGGL(k_slq_lds, dim3((unsigned)((P + PB - 1) / PB)), dim3(64),
                       (size_t)(24 * PB * Um), st, s.gam, s.xi, s.iters, g.T, g.C, K, g.Rp,
                       pnorm2, tau, ok, rmin, rmax, (int)PB, (int)Um);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_slq, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, s.gam, s.xi,
                     s.iters, g.T, g.C, K, g.Rp, pnorm2, dg, of, zz, tau, ok, rmin, rmax);
  return hipGetLastError();
}

}  // namespace cmtcs
