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
#include <type_traits>

#include "internal.h"

namespace cmtcs {

// Reciprocal square root of r2 > 0 for the Givens rotations.  On the device: the hardware
// estimate y0 refined by one third-order step, y = y0 (1 + e/2 + 3 e^2/8) with
// e = 1 - r2 y0^2 (the series of (1 - e)^(-1/2)), which cubes the relative error of the
// estimate; four dependent operations where two Newton steps take six, and the rotation's
// dependent chain is what bounds this kernel.
struct RsqDevice {
  __device__ double operator()(double r2) const {
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    const double p = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y0 * e, p, y0);
  }
};
// The same on the host (for host builds of this routine, which the tests compile).
struct RsqHost {
  __host__ double operator()(double r2) const { return 1.0 / std::sqrt(r2); }
};

// Eigenvalues (left in dg) and first eigenvector components (left in zz, which must enter as
// e_1) of the symmetric tridiagonal with diagonal dg[0..n-1] and off-diagonal of[0..n-2];
// element i of each array is at index i * stride (index type I: int for on-chip arrays).
// Each array must provide n + 1 entries: entry n (and of[n-1]) is scratch that a sweep may read
// ahead or write and never uses.  Returns 0 on success, 1 if the sweep limit was reached.
//
// The routine runs one probe per thread, and a wave executes the union of its lanes' control
// paths, so every branch is kept short: the bottom deflations run in their own small loop (so
// that each round of the outer loop is one sweep for every lane that is not done), the scan for
// the block start tests four off-diagonals per round, and the rotation loop has no branch.
template <typename I, typename Rsq>
__host__ __device__ inline int tridiag_eig_first_row(double* dg, double* of, double* zz, int n,
                                                     I stride, int max_sweeps, Rsq rsq) {
  const double eps = 2.220446049250313e-16;
  // off-diagonal j is negligible against its two diagonal neighbours
  auto small = [&](int j) __attribute__((always_inline)) {
    return fabs(of[(I)j * stride]) <=
           eps * (fabs(dg[(I)j * stride]) + fabs(dg[(I)(j + 1) * stride]));
  };
  int hi = n - 1;
  int sweeps = 0;
  while (true) {
    while (hi > 0 && small(hi - 1)) {
      of[(I)(hi - 1) * stride] = 0.0;
      --hi;
    }
    if (hi <= 0) break;
    // start of the unreduced block that ends at hi
    int lo = hi - 1;
    while (lo >= 4) {
      const bool s1 = small(lo - 1), s2 = small(lo - 2), s3 = small(lo - 3), s4 = small(lo - 4);
      if (s1 || s2 || s3 || s4) break;
      lo -= 4;
    }
    while (lo > 0 && !small(lo - 1)) --lo;
    if (lo > 0) of[(I)(lo - 1) * stride] = 0.0;
    if (++sweeps > max_sweeps) return 1;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer its last diagonal entry
    const double a = dg[(I)(hi - 1) * stride], bq = of[(I)(hi - 1) * stride];
    const double cq = dg[(I)hi * stride];
    const double delta = 0.5 * (a - cq);
    const double den = delta + copysign(hypot(delta, bq), delta);
    const double mu = cq - bq * bq / den;
    // Bulge chase: rotations in planes (k, k+1), k = lo..hi-1.  Rotation k writes positions
    // k-1 and k only, so the untouched entries at k+2 that the next rotation needs are loaded
    // one rotation ahead (up to position hi+1 <= n, the scratch entry at the end); the
    // off-diagonal read past the block end only feeds values the last rotation discards.  The
    // first rotation is peeled: it has no finished off-diagonal to store.
    double a0 = dg[(I)lo * stride], b0 = of[(I)lo * stride], z0 = zz[(I)lo * stride];
    double a1 = dg[(I)(lo + 1) * stride], z1 = zz[(I)(lo + 1) * stride];
    double b1 = of[(I)(lo + 1) * stride];
    double x = a0 - mu;
    double y = b0;
    auto rotate = [&](int k, auto first) __attribute__((always_inline)) {
      const double a2 = dg[(I)(k + 2) * stride], z2 = zz[(I)(k + 2) * stride];
      const double b2 = of[(I)(k + 2) * stride];
      // Givens rotation (cs, sn) = (x, y) / r zeroing y against x.  The entries are
      // eigenvalue-sized (CG step sizes of a positive definite system), far from FP64
      // overflow, so r needs no scaling.  The next x, the new off-diagonal
      //   nb = cs sn (a1 - a0) + (cs^2 - sn^2) b0 = [x y (a1 - a0) + (x - y)(x + y) b0] / r^2,
      // takes its bracket from values known before the rotation, so that the chain from one
      // rotation's x to the next runs through r^2, one reciprocal square root and two
      // products only.  r2 = 0 (x = y = 0) keeps the identity rotation.
      const double r2 = x * x + y * y;
      const double num = (x * y) * (a1 - a0) + ((x - y) * (x + y)) * b0;
      const double inv = rsq(fmax(r2, 1e-300));
      const double cs = r2 > 0.0 ? x * inv : 1.0;
      const double sn = y * inv;   // y = 0 when r2 = 0
      if constexpr (!decltype(first)::value) of[(I)(k - 1) * stride] = r2 * inv;
      const double nb = (num * inv) * inv;
      const double na0 = cs * cs * a0 + 2.0 * cs * sn * b0 + sn * sn * a1;
      const double na1 = sn * sn * a0 - 2.0 * cs * sn * b0 + cs * cs * a1;
      dg[(I)k * stride] = na0;
      of[(I)k * stride] = nb;
      zz[(I)k * stride] = cs * z0 + sn * z1;
      z0 = -sn * z0 + cs * z1;
      a0 = na1;
      y = (y * inv) * b1;   // bulge at (k+2, k): sn b1
      b0 = cs * b1;         // off-diagonal (k+1, k+2) after this rotation
      x = nb;
      a1 = a2; z1 = z2; b1 = b2;
    };
    rotate(lo, std::true_type{});
    for (int k = lo + 1; k < hi; ++k) rotate(k, std::false_type{});
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
// thread each), arrays laid out [u][probe] in dynamic shared memory of 3 * PB * (Um + 1)
// doubles.
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
  // Um + 1 positions per array: the eigensolver's scratch entry follows the last step
  double* dg = sm + lp;
  double* of = sm + (long)PB * (Um + 1) + lp;
  double* zz = sm + 2L * PB * (Um + 1) + lp;
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
  // A wave pays for every instruction whatever number of its lanes hold a probe, and one wave
  // per SIMD leaves the long dependent chains of its rotations exposed.  27 KB of LDS per
  // one-wave block balances the two: at 200 steps, 5 probes per wave and six blocks per CU
  // (measured at 8192 probes: 22 ms, against 25 ms at 20 KB, 29 ms at 40 KB and 36 ms at 10 KB).
  // With many probes (more than fit on chip in one round), one probe per lane in full waves
  // with the global-memory layout needs fewer rounds and wins.
  constexpr long kLdsBytes = 27 * 1024;
  constexpr long kLdsMaxProbes = 16384;
  const long Um = steps > 0 ? steps : 1;
  const long PB = std::min<long>(64, kLdsBytes / (24 * (Um + 1)));
  if (PB >= 1 && P <= kLdsMaxProbes) {
    hipLaunchKernelGGL(k_slq_lds, dim3((unsigned)((P + PB - 1) / PB)), dim3(64),
                       (size_t)(24 * PB * (Um + 1)), st, s.gam, s.xi, s.iters, g.T, g.C, K, g.Rp,
                       pnorm2, tau, ok, rmin, rmax, (int)PB, (int)Um);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_slq, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, s.gam, s.xi,
                     s.iters, g.T, g.C, K, g.Rp, pnorm2, dg, of, zz, tau, ok, rmin, rmax);
  return hipGetLastError();
}

}  // namespace cmtcs
