// EM pieces around the batched solves (Alg. 2): the mean right-hand side b_t = beta Phi_t^T y_t
// (Eq. (lin-sys)), the responsibilities q_tc (Eq. (estep)) and the alpha update (Eq. (mstep)).
// All sums are FP64 in a fixed order.
#include "internal.h"

namespace cmtcs {

// b_t[d] = beta sum_n Phi_t[n][d] y_t[n]: one thread per (t, d), rows read coalesced.
template <typename VT>
__global__ __launch_bounds__(256) void k_rhs(const float* __restrict__ phi,
                                             const int64_t* __restrict__ row_off,
                                             const float* __restrict__ y, double beta,
                                             VT* __restrict__ b, int D) {
  const int t = blockIdx.x;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  const int64_t r0 = row_off[t], r1 = row_off[t + 1];
  double acc = 0.0;
  for (int64_t n = r0; n < r1; ++n) acc += (double)phi[n * D + d] * (double)y[n];
  b[(int64_t)t * D + d] = (VT)(beta * acc);
}

// const_t = -(n_t / 2) log(2 pi) + (n_t / 2) log beta - (beta / 2) y_t . y_t over the task's n_t
// real measurements (per_row = 1 per stored row, 2 for (re, im) pairs), one block per task:
// ell_tc / 2 + const_t is then log N(y_t; 0, beta^-1 I + Phi_t diag(alpha_c)^-1 Phi_t^T)
// (Sec. 2).
__global__ __launch_bounds__(256) void k_log_norm_const(const float* __restrict__ y,
                                                        const int64_t* __restrict__ row_off,
                                                        int per_row, double beta,
                                                        double* __restrict__ lconst) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  const int64_t i0 = row_off[t] * per_row, i1 = row_off[t + 1] * per_row;
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += (double)y[i] * (double)y[i];
  const double yy = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) {
    const double n = (double)(i1 - i0);
    lconst[t] = -0.5 * n * log(2.0 * 3.14159265358979323846) + 0.5 * n * log(beta) - 0.5 * beta * yy;
  }
}

// L_t = log sum_c exp(ell_tc / 2 + log pi_c) + const_t (max-shifted) and their mean Lhat, one
// block; the mean is a fixed-order sum.
__global__ __launch_bounds__(256) void k_log_likelihood(const double* __restrict__ ell,
                                                        const double* __restrict__ log_pi,
                                                        const double* __restrict__ lconst,
                                                        int T, int C, double* __restrict__ Lt,
                                                        double* __restrict__ L) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int t = threadIdx.x; t < T; t += 256) {
    double m = -INFINITY;
    for (int c = 0; c < C; ++c) m = fmax(m, 0.5 * ell[(int64_t)t * C + c] + log_pi[c]);
    double sum = 0.0;
    for (int c = 0; c < C; ++c) sum += exp(0.5 * ell[(int64_t)t * C + c] + log_pi[c] - m);
    // a non-finite ell (a failed task) propagates instead of being skipped by fmax
    bool bad = false;
    for (int c = 0; c < C; ++c) bad = bad || !isfinite(ell[(int64_t)t * C + c]);
    const double v = bad ? NAN : m + log(sum) + lconst[t];
    if (Lt != nullptr) Lt[t] = v;
    acc += v;
  }
  const double tot = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && L != nullptr) *L = tot / (double)T;
}

hipError_t launch_log_norm_const(int T, const float* y, const int64_t* row_off, int per_row,
                                 double beta, double* lconst, hipStream_t st) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_log_norm_const, dim3(T), dim3(256), 0, st, y, row_off, per_row, beta,
                     lconst);
  return hipGetLastError();
}

hipError_t launch_log_likelihood(int T, int C, const double* ell, const double* log_pi,
                                 const double* lconst, double* Lt, double* L, hipStream_t st) {
  hipLaunchKernelGGL(k_log_likelihood, dim3(1), dim3(256), 0, st, ell, log_pi, lconst, T, C, Lt,
                     L);
  return hipGetLastError();
}

// sum_d log alpha_cd, one block per cluster.
__global__ __launch_bounds__(256) void k_sum_log_alpha(const float* __restrict__ alpha,
                                                       double* __restrict__ slog, int D) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int d = threadIdx.x; d < D; d += 256) acc += log((double)alpha[(int64_t)c * D + d]);
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) slog[c] = s;
}

// Per task t (one block):
//   nu_tc  = -(1/K') sum_k tau_tck over the K' probes with a positive spectrum (Eq. (logdet-est))
//   ell_tc = nu_tc + sum_d log alpha_cd + b_t . mu_tc   (Eq. (estep): beta y^T Phi mu = b . mu)
//   q_tc   = softmax over c of z_tc = ell_tc / 2 + log pi_c
template <typename VT>
__global__ __launch_bounds__(256) void k_resp(const VT* __restrict__ X, const VT* __restrict__ b,
                                              const double* __restrict__ tau,
                                              const uint8_t* __restrict__ ok,
                                              const double* __restrict__ slog,
                                              const double* __restrict__ log_pi,
                                              double* __restrict__ logdet,
                                              double* __restrict__ ell, double* __restrict__ q,
                                              int* __restrict__ keff_out,
                                              const double* __restrict__ slogm, int C, int K,
                                              int Rp, int D) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  const VT* bt = b + (int64_t)t * D;
  for (int c = 0; c < C; ++c) {
    const VT* mu = X + ((int64_t)t * Rp + (int64_t)c * (K + 1)) * D;
    double acc = 0.0;
    for (int d = threadIdx.x; d < D; d += 256) acc += (double)bt[d] * (double)mu[d];
    const double dot = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) {
      double st = 0.0;
      int keff = 0;
      for (int k = 0; k < K; ++k) {
        const int64_t p = ((int64_t)t * C + c) * K + k;
        if (ok[p]) { st += tau[p]; ++keff; }
      }
      // Jacobi preconditioning: the quadrature estimates log det of M^-1/2 A M^-1/2, and
      // log det A = sum_d log M_dd + that
      const double corr = slogm != nullptr ? slogm[(int64_t)t * C + c] : 0.0;
      const double nu = keff > 0 ? -st / (double)keff - corr : NAN;
      keff_out[(int64_t)t * C + c] = keff;
      logdet[(int64_t)t * C + c] = nu;
      ell[(int64_t)t * C + c] = nu + slog[c] + dot;
    }
  }
  if (threadIdx.x == 0) {
    double m = -INFINITY;
    for (int c = 0; c < C; ++c) m = fmax(m, 0.5 * ell[(int64_t)t * C + c] + log_pi[c]);
    // q_c = exp(z_c - m) / sum_c' exp(z_c' - m): the same softmax as exp(z_c - logsumexp z),
    // normalised by a division so that the q of a task sum to 1 within a few roundings even
    // when |z| is large
    double se = 0.0;
    for (int c = 0; c < C; ++c) se += exp(0.5 * ell[(int64_t)t * C + c] + log_pi[c] - m);
    for (int c = 0; c < C; ++c)
      q[(int64_t)t * C + c] = exp(0.5 * ell[(int64_t)t * C + c] + log_pi[c] - m) / se;
  }
}

// alpha_cd = Nq_c / den_cd with the guards stated in the ABI header; one thread per (c, d).
// A task whose q_tc is not finite (e.g. every probe of (t, c) excluded from nu, so that q_t is
// NaN) is left out of cluster c's sums; a denominator that is still not finite (a non-finite mu
// or s entry) keeps the old alpha_cd.
__global__ __launch_bounds__(256) void k_mstep(const float* __restrict__ mu,
                                               const float* __restrict__ sdiag,
                                               const double* __restrict__ q, double alpha_max,
                                               float* __restrict__ alpha, int T, int C, int D) {
  const int c = blockIdx.y;
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= D) return;
  double nq = 0.0, den = 0.0;
  for (int t = 0; t < T; ++t) {
    const double w = q[(int64_t)t * C + c];
    if (!isfinite(w)) continue;
    const int64_t i = ((int64_t)t * C + c) * D + d;
    const double m = (double)mu[i];
    nq += w;
    den += w * (m * m + (double)sdiag[i]);
  }
  if (nq < 1e-300 || !isfinite(den)) return;
  alpha[(int64_t)c * D + d] = den > nq / alpha_max ? (float)(nq / den) : (float)alpha_max;
}

// log pi_c = log((1/T) sum_t q_tc): the mixture-weight M-step when the cluster weights are
// learned rather than given (Sec. 2).  One thread per cluster, sum in task order; a cluster with
// no mass gets -inf.
__global__ __launch_bounds__(64) void k_update_pi(const double* __restrict__ q,
                                                  double* __restrict__ log_pi, int T, int C) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= C) return;
  double nq = 0.0;
  for (int t = 0; t < T; ++t) nq += q[(int64_t)t * C + c];
  log_pi[c] = log(nq / (double)T);
}

template <typename VT>
hipError_t launch_rhs(const Geometry& g, const float* phi, const float* y, double beta, VT* b,
                      hipStream_t st) {
  hipLaunchKernelGGL((k_rhs<VT>), dim3(g.T, (g.D + 255) / 256), dim3(256), 0, st, phi,
                     g.row_off, y, beta, b, g.D);
  return hipGetLastError();
}

hipError_t launch_sum_log_alpha(int C, int D, const float* alpha, double* slog, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_log_alpha, dim3(C), dim3(256), 0, st, alpha, slog, D);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_resp(const Geometry& g, const CgState& s, int K, const VT* b,
                       const double* tau, const uint8_t* ok, const double* slog,
                       const double* log_pi, double* logdet, double* ell, double* q,
                       int* keff, const double* slogm, hipStream_t st) {
  hipLaunchKernelGGL((k_resp<VT>), dim3(g.T), dim3(256), 0, st, (const VT*)s.X, b, tau, ok, slog,
                     log_pi, logdet, ell, q, keff, slogm, g.C, K, g.Rp, g.D);
  return hipGetLastError();
}

hipError_t launch_mstep(int T, int C, int D, const float* mu, const float* sdiag,
                        const double* q, double alpha_max, float* alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_mstep, dim3((D + 255) / 256, C), dim3(256), 0, st, mu, sdiag, q,
                     alpha_max, alpha, T, C, D);
  return hipGetLastError();
}

hipError_t launch_update_pi(int T, int C, const double* q, double* log_pi, hipStream_t st) {
  hipLaunchKernelGGL(k_update_pi, dim3((C + 63) / 64), dim3(64), 0, st, q, log_pi, T, C);
  return hipGetLastError();
}

template hipError_t launch_rhs<double>(const Geometry&, const float*, const float*, double,
                                       double*, hipStream_t);
template hipError_t launch_rhs<float>(const Geometry&, const float*, const float*, double,
                                      float*, hipStream_t);
template hipError_t launch_resp<double>(const Geometry&, const CgState&, int, const double*,
                                        const double*, const uint8_t*, const double*,
                                        const double*, double*, double*, double*, int*,
                                        const double*, hipStream_t);
template hipError_t launch_resp<float>(const Geometry&, const CgState&, int, const float*,
                                       const double*, const uint8_t*, const double*,
                                       const double*, double*, double*, double*, int*,
                                       const double*, hipStream_t);

}  // namespace cmtcs
