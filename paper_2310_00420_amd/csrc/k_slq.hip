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
// The sum is e_1^T log(Gamma-bar) e_1.  It is computed here without an eigendecomposition, from
// log x = int_0^inf [1/(1+t) - 1/(x+t)] dt (x > 0) applied to the spectrum:
//     sum_u S_{u,1}^2 log lambda_u = int_0^inf [1/(1+t) - e_1^T (Gamma-bar + t I)^{-1} e_1] dt.
// With t = e^s the integrand is analytic in the strip |Im s| < pi (its poles sit at
// s = log lambda_u +- i pi and +- i pi) and decays like e^{-|s|} outside
// [min(log lambda_min, 0), max(log lambda_max, 0)], so the trapezoidal rule with step h on that
// interval widened by L on each side has error of order exp(-2 pi^2 / h) + e^{-L}: h = 0.45 and
// L = 36 give about 1e-14 relative (against LAPACK's eigendecomposition, tridiagonals of
// condition up to 1e8).  The resolvent entry is Q_1 / Q_0, Q_u being the determinant of the
// trailing block (rows u..U-1) of Gamma-bar + t I, from the three-term recurrence
// Q_u = (a_u + t) Q_{u+1} - b_u^2 Q_{u+2} run from the bottom without divisions and rescaled by
// powers of two; the integrand is then t ((a_0 - 1) Q_1 - b_0^2 Q_2) / ((1 + t) Q_0), in which
// the two O(1) terms that cancel for large t have already been subtracted exactly.
//
// lambda_min and lambda_max (the interval above, and outputs) come from Sturm counts: for
// Gamma-bar - x I the number of negative pivots Q_u / Q_{u+1} equals the number of eigenvalues
// below x (Sylvester's law of inertia applied to the U D U^T factorisation).  They are as
// accurate as bisection, i.e. to about eps * ||Gamma-bar|| in absolute terms.
//
// Every quadrature node and every Sturm point is independent of the others, so one wave
// handles one probe: its 64 lanes share the two searches (32 points per end and round) and then
// the nodes, with the probe's U rows in LDS read by all lanes at once.  All loops have trip
// counts fixed by U and the round count, whatever the data.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "internal.h"

namespace cmtcs {

// Row u of Gamma-bar: diagonal entry and squared off-diagonal to row u + 1 (0 for the last).
struct alignas(16) TriRow {
  double a, b2;
};

// Multiplies x and y by the power of two that brings the larger magnitude into [0.5, 1).
struct ScaleDevice {
  __device__ void operator()(double& x, double& y) const {
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(x), fabs(y)));
    x = __builtin_amdgcn_ldexp(x, -e);
    y = __builtin_amdgcn_ldexp(y, -e);
  }
};
// The same on the host (for host builds of these routines, which the tests compile).
struct ScaleHost {
  __host__ void operator()(double& x, double& y) const {
    int e = 0;
    (void)std::frexp(std::fmax(std::fabs(x), std::fabs(y)), &e);
    x = std::ldexp(x, -e);
    y = std::ldexp(y, -e);
  }
};

constexpr double kQuadStep = 0.45;    // h
constexpr double kQuadTail = 36.0;    // L
constexpr int kSecPoints = 32;        // Sturm points per end and round
constexpr int kSecRounds = 11;        // (kSecPoints + 1)^11 = 5e16: the bracket reaches rounding

// Q_1 and Q_2 of Gamma-bar + t I (rows r[0..n-1], n >= 1, at one common power-of-two scale)
// by the recurrence from the bottom; with kCount, also the number of negative pivots
// Q_u / Q_{u+1} for u = n-1..1 (a zero pivot is replaced by a tiny negative one, as in
// bisection codes, so that the next pivot stays finite).  Rescaled after every fourth row: a
// row changes the magnitude of the pair by a factor between its off-diagonal squared and
// |a + t| + b^2, well within the exponent range for four rows.
template <bool kCount, typename Rows, typename Scale>
__host__ __device__ inline int trailing_det(const Rows& r, int n, double t, double& q1, double& q2,
                                            Scale sc) {
  double x1 = 1.0, x2 = 0.0;   // Q_{u+1}, Q_{u+2}
  int neg = 0;
  auto row = [&](const TriRow w) __attribute__((always_inline)) {
    double q = std::fma(w.a + t, x1, -(w.b2 * x2));
    if (kCount) {
      if (q == 0.0) q = -0x1p-80 * x1;
      neg += (q < 0.0) != (x1 < 0.0);
    }
    x2 = x1;
    x1 = q;
  };
  int u = n - 1;
  for (; u >= 4; u -= 4) {
    const TriRow w0 = r[u], w1 = r[u - 1], w2 = r[u - 2], w3 = r[u - 3];   // loads together
    row(w0);
    row(w1);
    row(w2);
    row(w3);
    sc(x1, x2);
  }
  for (; u >= 1; --u) row(r[u]);
  q1 = x1;
  q2 = x2;
  return neg;
}

// Number of eigenvalues of Gamma-bar below x (negative pivots of Gamma-bar - x I).
template <typename Rows, typename Scale>
__host__ __device__ inline int sturm_count(const Rows& r, int n, double x, Scale sc) {
  double q1, q2;
  int neg = trailing_det<true>(r, n, -x, q1, q2, sc);
  double q0 = std::fma(r[0].a - x, q1, -(r[0].b2 * q2));
  if (q0 == 0.0) q0 = -0x1p-80 * q1;
  return neg + ((q0 < 0.0) != (q1 < 0.0));
}

// Integrand at s (t = e^s): t [1/(1+t) - e_1^T (Gamma-bar + t I)^{-1} e_1].
template <typename Rows, typename Scale>
__host__ __device__ inline double quad_node(const Rows& r, int n, double s, Scale sc) {
  const double t = std::exp(s);
  double q1, q2;
  (void)trailing_det<false>(r, n, t, q1, q2, sc);
  const TriRow w = r[0];
  const double q0 = std::fma(w.a + t, q1, -(w.b2 * q2));
  return t * std::fma(w.a - 1.0, q1, -(w.b2 * q2)) / ((1.0 + t) * q0);
}

// Nodes s_j = s0 + j h, j < nodes, covering [min(log lo, 0) - L, max(log hi, 0) + L] for a
// spectrum inside [lo, hi], lo > 0.
__host__ __device__ inline void quad_range(double lo, double hi, double& s0, int& nodes) {
  s0 = std::fmin(std::log(lo), 0.0) - kQuadTail;
  const double s1 = std::fmax(std::log(hi), 0.0) + kQuadTail;
  nodes = (int)std::ceil((s1 - s0) / kQuadStep) + 1;
}

// Point k (1..kSecPoints) of a bracket split into kSecPoints + 1 parts, and the bracket after a
// round given the points that reached the count sought (bit k-1 of hit): from the last point
// below the first hit to the first hit (the ends of the old bracket where there is none).
__host__ __device__ inline double sec_point(double lo, double hi, int k) {
  return lo + (hi - lo) * (double)k * (1.0 / (kSecPoints + 1));
}
__host__ __device__ inline void sec_update(double& lo, double& hi, uint32_t hit) {
  const int k = hit ? __builtin_ctz(hit) + 1 : kSecPoints + 1;
  const double nlo = k > 1 ? sec_point(lo, hi, k - 1) : lo;
  const double nhi = k <= kSecPoints ? sec_point(lo, hi, k) : hi;
  lo = nlo;
  hi = nhi;
}

// Starting bracket for both ends: the Gershgorin interval, widened by a margin well above the
// rounding of the Sturm counts.
__host__ __device__ inline void sec_start(double& glo, double& ghi) {
  const double m = std::ldexp(std::fmax(std::fabs(glo), std::fabs(ghi)), -40) + 1e-300;
  glo -= m;
  ghi += m;
}

template <typename VT>
__device__ inline VT wave_sum(VT v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One wave per probe, W = blockDim.x / 64 probes per block.  kLds: the rows live in dynamic LDS
// (Um rows per wave); otherwise in the workspace rows_ws, Um rows per probe.
template <bool kLds>
__global__ __launch_bounds__(256) void k_slq(const double* __restrict__ gam,
                                             const double* __restrict__ xi,
                                             const int* __restrict__ iters, int T, int C,
                                             int K, int Rp, double pnorm2, int Um,
                                             TriRow* __restrict__ rows_ws,
                                             double* __restrict__ tau,
                                             uint8_t* __restrict__ ok,
                                             double* __restrict__ rmin,
                                             double* __restrict__ rmax) {
  extern __shared__ TriRow sm_rows[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long P = (long)T * C * K;
  const long p = (long)blockIdx.x * (blockDim.x >> 6) + wv;
  long idx = 0;
  int n = 0;
  if (p < P) {
    const int t = (int)(p / ((long)C * K));
    const int c = (int)((p / K) % C);
    const int k = (int)(p % K);
    idx = (long)t * Rp + (long)c * (K + 1) + 1 + k;
    n = iters[idx];
  }
  n = __builtin_amdgcn_readfirstlane(n);
  TriRow* r = kLds ? sm_rows + (long)wv * Um : rows_ws + (p < P ? p : 0) * (long)Um;
  const long ncol = (long)T * Rp;
  // rows of Gamma-bar (Eq. (tridiag)) and the Gershgorin interval
  double glo = INFINITY, ghi = -INFINITY;
  bool finite = true;
  for (int u = lane; u < n; u += 64) {
    const double g = gam[(long)u * ncol + idx];
    double a = 1.0 / g, bu = 0.0, bl = 0.0;
    if (u > 0) {
      const double gp = gam[(long)(u - 1) * ncol + idx];
      const double xp = xi[(long)(u - 1) * ncol + idx];
      a += xp / gp;
      bl = sqrt(xp) / gp;
    }
    TriRow w{a, 0.0};
    if (u + 1 < n) {
      const double x = xi[(long)u * ncol + idx];
      w.b2 = x / (g * g);
      bu = sqrt(x) / g;
    }
    r[u] = w;
    glo = fmin(glo, a - bl - bu);
    ghi = fmax(ghi, a + bl + bu);
    finite = finite && isfinite(a) && isfinite(w.b2);
  }
  // the rows are read by every lane of the wave: a block barrier for LDS, a device-scope fence
  // (stores completed, caches made coherent) for the workspace
  if (kLds) __syncthreads();
  else __threadfence();
  if (n == 0) {
    if (p < P && lane == 0) { tau[p] = 0.0; ok[p] = 0; rmin[p] = NAN; rmax[p] = NAN; }
    return;
  }
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  const bool all_finite = __all(finite);
  if (!all_finite) {
    if (lane == 0) { tau[p] = 0.0; ok[p] = 0; rmin[p] = NAN; rmax[p] = NAN; }
    return;
  }
  sec_start(glo, ghi);
  // multisection: lanes 0..31 search lambda_min (first point with a count >= 1), lanes 32..63
  // lambda_max (first point with a count >= n)
  const int end = lane >> 5, kp = (lane & 31) + 1;
  const int want = end ? n : 1;
  double lo = glo, hi = ghi;
  for (int it = 0; it < kSecRounds; ++it) {
    const int cnt = sturm_count(r, n, sec_point(lo, hi, kp), ScaleDevice());
    const uint64_t hit = __ballot(cnt >= want);
    sec_update(lo, hi, end ? (uint32_t)(hit >> 32) : (uint32_t)hit);
  }
  const double lmin_lo = __shfl(lo, 0, 64), lmin_hi = __shfl(hi, 0, 64);
  const double lmax_lo = __shfl(lo, 32, 64), lmax_hi = __shfl(hi, 32, 64);
  // positive definite: no eigenvalue at or below the lower end of lambda_min's bracket
  const bool pd = lmin_lo > 0.0;
  double acc = 0.0;
  if (pd) {
    double s0;
    int nodes;
    quad_range(lmin_lo, lmax_hi, s0, nodes);
    for (int j0 = 0; j0 < nodes; j0 += 64) {
      const int j = j0 + lane;
      const double f = quad_node(r, n, s0 + (double)(j < nodes ? j : 0) * kQuadStep,
                                 ScaleDevice());
      acc += j < nodes ? f : 0.0;
    }
    acc = wave_sum(acc) * kQuadStep;
  }
  if (lane == 0) {
    tau[p] = pd ? pnorm2 * acc : 0.0;
    ok[p] = pd ? 1 : 0;
    rmin[p] = 0.5 * (lmin_lo + lmin_hi);
    rmax[p] = 0.5 * (lmax_lo + lmax_hi);
  }
}

// Four probes (waves) per block while their rows fit in the LDS budget (kSlqLdsBytes unless
// a smaller one is given), fewer for long runs, and the workspace beyond one wave's worth.
static long slq_waves(long Um, long lds_bytes) {
  return std::min<long>(4, lds_bytes / (long)(sizeof(TriRow) * Um));
}

size_t slq_workspace_bytes(long P, int steps, long lds_bytes) {
  const long Um = steps > 0 ? steps : 1;
  return slq_waves(Um, lds_bytes) >= 1 ? 0 : sizeof(TriRow) * (size_t)P * (size_t)Um;
}

hipError_t launch_slq(const Geometry& g, const CgState& s, int K, int steps, double pnorm2,
                      void* rows_ws, double* tau, uint8_t* ok, double* rmin, double* rmax,
                      long lds_bytes, hipStream_t st) {
  const long P = (long)g.T * g.C * K;
  if (P == 0) return hipSuccess;
  const long Um = steps > 0 ? steps : 1;
  const long W = slq_waves(Um, lds_bytes);
  if (W >= 1) {
    hipLaunchKernelGGL(k_slq<true>, dim3((unsigned)((P + W - 1) / W)), dim3((unsigned)(64 * W)),
                       (size_t)(sizeof(TriRow) * W * Um), st, s.gam, s.xi, s.iters, g.T, g.C, K,
                       g.Rp, pnorm2, (int)Um, (TriRow*)rows_ws, tau, ok, rmin, rmax);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_slq<false>, dim3((unsigned)P), dim3(64), 0, st, s.gam, s.xi, s.iters, g.T,
                     g.C, K, g.Rp, pnorm2, (int)Um, (TriRow*)rows_ws, tau, ok, rmin, rmax);
  return hipGetLastError();
}

}  // namespace cmtcs
