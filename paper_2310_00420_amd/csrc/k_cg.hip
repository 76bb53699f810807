// Conjugate gradient (Alg. 1) over every right-hand side of every task at once (Sec. 3.3), and
// the estimators read straight off the CG solutions: the posterior mean mu_tc (the mean system
// of Eq. (lin-sys)) and the diagonal estimate s_tc = (1/K) sum_k p_k (.) x_k (Eq. (diag-est)).
//
// One workgroup owns one right-hand side (a column of D elements, held in registers), so both
// reductions of a CG step (d.Ad and the new r.r) finish inside the workgroup and the whole
// vector update of Alg. 1 (gamma, x, r, xi, d) is a single kernel.  Scalars are FP64 and the
// reduction order is fixed, so results are identical run to run.
#include <algorithm>

#include "internal.h"
#include "../../include/cmtcs.h"

namespace cmtcs {

// PC: Jacobi-preconditioned start (mdiag = M = diag(A_tc) per (t, c)): probe right-hand sides
// are M^1/2 p, z = M^-1 r, d = z, rr holds r.z, and thr is tol^2 ||b||^2 on the plain residual.
template <typename VT, int BS, int EPT, bool PC>
__global__ __launch_bounds__(BS) void k_cg_init(VT* __restrict__ X, VT* __restrict__ Rv,
                                                VT* __restrict__ Dv, double* __restrict__ rr,
                                                double* __restrict__ thr,
                                                uint8_t* __restrict__ state,
                                                int* __restrict__ iters, int* __restrict__ act,
                                                int kind, const VT* __restrict__ b,
                                                const VT* __restrict__ B, int K,
                                                const uint64_t* __restrict__ keyp,
                                                const int8_t* __restrict__ probes, double tol2,
                                                int C, int R, int Rp, int D, int crn,
                                                const double* __restrict__ mdiag,
                                                const int* __restrict__ colc) {
  __shared__ double sh[2 * (BS / 64)];
  const int col = blockIdx.x;
  const int t = col / Rp, j = col % Rp;
  const int64_t base = (int64_t)col * D;
  if (j >= R) {   // padding slot: keep it zero so the operator products see zero columns
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = threadIdx.x + e * BS;
      if (d < D) { X[base + d] = 0; Rv[base + d] = 0; Dv[base + d] = 0; }
    }
    return;
  }
  int c = 0, k = 0;
  uint64_t key = 0;
  if (kind == 0) {
    c = j / (K + 1);
    k = j % (K + 1);
    if (probes == nullptr) key = *keyp;
  }
  const double* mcol = nullptr;
  if constexpr (PC) mcol = mdiag + ((int64_t)t * C + (kind == 0 ? c : colc[col])) * D;
  double acc = 0.0, accz = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int d = threadIdx.x + e * BS;
    if (d >= D) continue;
    VT v;
    if (kind == 0) {
      if (k == 0) v = b[(int64_t)t * D + d];
      else {
        double pv = probes != nullptr
                        ? (double)probes[(((int64_t)t * C + c) * K + (k - 1)) * D + d]
                        : probe_entry(key, t, crn ? 0 : c, k - 1, d, C, K, D);
        if constexpr (PC) pv *= sqrt(mcol[d]);
        v = (VT)pv;
      }
    } else {
      v = B[((int64_t)t * R + j) * D + d];
    }
    X[base + d] = 0;
    Rv[base + d] = v;
    if constexpr (PC) {
      const VT z = (VT)((double)v / mcol[d]);
      Dv[base + d] = z;
      accz += (double)v * (double)z;
    } else {
      Dv[base + d] = v;
    }
    acc += (double)v * (double)v;
  }
  double r0, rz0;
  if constexpr (PC) {
    const d2 sums = block_sum2<BS>(acc, accz, sh);
    r0 = sums[0];
    rz0 = sums[1];
  } else {
    r0 = block_sum<BS>(acc, sh);
    rz0 = r0;
  }
  if (threadIdx.x == 0) {
    rr[col] = rz0;
    thr[col] = tol2 * r0;
    iters[col] = 0;
    uint8_t st;
    if (!isfinite(r0)) st = CMTCS_CG_BREAKDOWN;
    else if (r0 > 0.0) st = kActive;
    else st = CMTCS_CG_CONVERGED;   // b = 0: x = 0 is exact
    state[col] = st;
    if (st == kActive) atomicAdd(&act[t], 1);
  }
}

// One step u of Alg. 1 for every active right-hand side (Alg. 1, lines 3-7):
//   gamma = r.r / d.Ad;  x += gamma d;  r -= gamma Ad;  xi = r'.r' / r.r;  d = r' + xi d.
// PC (Jacobi, z = M^-1 r): gamma = r.z / d.Ad, xi = r'.z' / r.z, d = z' + xi d; the stop rule
// tests r'.r'.
template <typename VT, int BS, int EPT, bool PC>
__global__ __launch_bounds__(BS) void k_cg_update(VT* __restrict__ X, VT* __restrict__ Rv,
                                                  VT* __restrict__ Dv,
                                                  const VT* __restrict__ AD,
                                                  double* __restrict__ rr,
                                                  const double* __restrict__ thr,
                                                  uint8_t* __restrict__ state,
                                                  int* __restrict__ iters,
                                                  double* __restrict__ gam,
                                                  double* __restrict__ xi, int* __restrict__ act,
                                                  int u, int steps, int fixed, int T, int R,
                                                  int Rp, int D, int split,
                                                  const float* __restrict__ alpha,
                                                  const int* __restrict__ colc, double beta,
                                                  void* __restrict__ d16, int d16_kind,
                                                  int64_t d16_ld,
                                                  const double* __restrict__ mdiag, int C) {
  __shared__ double sh[2 * (BS / 64)];
  const int t = blockIdx.x / R, j = blockIdx.x % R;
  const int64_t idx = (int64_t)t * Rp + j;
  if (state[idx] != kActive) return;
  const double rr_old = rr[idx];   // read by every thread before thread 0 rewrites it
  const int64_t base = idx * D;
  // with alpha given, AD holds Phi^T Phi d and A d = beta AD + alpha_c (.) d is formed here,
  // with the same fused multiply-add as the product's own epilogue
  const int c = alpha != nullptr ? colc[idx] : -1;
  const float* al = alpha + (int64_t)(c >= 0 ? c : 0) * D;
  // all four vectors are loaded before the first reduction so that the r and x loads are in
  // flight while d.Ad is summed.  With an even number of elements per thread, each thread
  // takes pairs of consecutive elements (one 2-wide load or store per vector and pair);
  // element e of a thread is d = el(e).
  // (not for 16 FP64 elements per thread, where the pairs cost more registers than there are)
  constexpr int P = EPT % 2 == 0 && !(sizeof(VT) == 8 && EPT >= 16) ? 2 : 1;
  typedef typename VecOf<VT, P>::type vp;
  auto el = [&](int e) __attribute__((always_inline)) {
    return P * ((int)threadIdx.x + (e / P) * BS) + e % P;
  };
  VT dv[EPT], av[EPT], rv[EPT], xv[EPT];
  double pd = 0.0;
#pragma unroll
  for (int e0 = 0; e0 < EPT; e0 += P) {
    const int d = el(e0);
    if (d < D) {   // D is a multiple of 16: a pair is in range with its first element
      vp x4[4];
      x4[0] = *(const vp*)(Dv + base + d);
      x4[1] = *(const vp*)(AD + base + d);
      x4[2] = *(const vp*)(Rv + base + d);
      x4[3] = *(const vp*)(X + base + d);
#pragma unroll
      for (int q = 0; q < P; ++q) {
        VT dq, aq, rq, xq;
        if constexpr (P == 1) { dq = x4[0]; aq = x4[1]; rq = x4[2]; xq = x4[3]; }
        else { dq = x4[0][q]; aq = x4[1][q]; rq = x4[2][q]; xq = x4[3][q]; }
        if (alpha != nullptr) {
          const VT a = c >= 0 ? (VT)al[d + q] : (VT)0;
          aq = __builtin_fma((VT)beta, aq, a * dq);
        }
        dv[e0 + q] = dq; av[e0 + q] = aq; rv[e0 + q] = rq; xv[e0 + q] = xq;
        pd += (double)dq * (double)aq;
      }
    } else {
#pragma unroll
      for (int q = 0; q < P; ++q) { dv[e0 + q] = 0; av[e0 + q] = 0; rv[e0 + q] = 0; xv[e0 + q] = 0; }
    }
  }
  const double dAd = block_sum<BS>(pd, sh);
  if (!(dAd > 0.0) || !isfinite(dAd)) {
    if (threadIdx.x == 0) state[idx] = CMTCS_CG_BREAKDOWN;
    return;
  }
  const double g = rr_old / dAd;
  const VT gv = (VT)g;
  double pr = 0.0;
  auto store = [&](VT* v, int e0, auto value) __attribute__((always_inline)) {
    vp o;
    if constexpr (P == 1) o = value(0);
    else { o[0] = value(0); o[1] = value(1); }
    *(vp*)(v + base + el(e0)) = o;
  };
#pragma unroll
  for (int e0 = 0; e0 < EPT; e0 += P) {
    if (el(e0) < D) {
      store(X, e0, [&](int q) { return xv[e0 + q] + gv * dv[e0 + q]; });
#pragma unroll
      for (int q = 0; q < P; ++q) {
        rv[e0 + q] = rv[e0 + q] - gv * av[e0 + q];
        pr += (double)rv[e0 + q] * (double)rv[e0 + q];
      }
    }
  }
  if (split) {
    // first half of a residual-replacement step: x and the recursive r only; the true
    // residual, xi, d and the stop decision follow in k_replace
#pragma unroll
    for (int e0 = 0; e0 < EPT; e0 += P)
      if (el(e0) < D) store(Rv, e0, [&](int q) { return rv[e0 + q]; });
    if (threadIdx.x == 0) gam[(int64_t)u * T * Rp + idx] = g;
    return;
  }
  double rrn, rzn;
  if constexpr (PC) {
    // z = M^-1 r' overwrites the copy of A d, no longer needed
    const double* mcol = mdiag + ((int64_t)t * C + colc[idx]) * D;
    double pz = 0.0;
#pragma unroll
    for (int e0 = 0; e0 < EPT; e0 += P) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int d = el(e0) + q;
        if (el(e0) < D) {
          av[e0 + q] = (VT)((double)rv[e0 + q] / mcol[d]);
          pz += (double)rv[e0 + q] * (double)av[e0 + q];
        }
      }
    }
    const d2 sums = block_sum2<BS>(pr, pz, sh);
    rrn = sums[0];
    rzn = sums[1];
  } else {
    rrn = block_sum<BS>(pr, sh);
    rzn = rrn;
  }
  const double x_ = rzn / rr_old;
  const VT xv_ = (VT)x_;
#pragma unroll
  for (int e0 = 0; e0 < EPT; e0 += P) {
    const int d = el(e0);
    if (d < D) {
      store(Rv, e0, [&](int q) { return rv[e0 + q]; });
      if constexpr (PC) store(Dv, e0, [&](int q) { return av[e0 + q] + xv_ * dv[e0 + q]; });
      else store(Dv, e0, [&](int q) { return rv[e0 + q] + xv_ * dv[e0 + q]; });
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const VT dn = (PC ? av[e0 + q] : rv[e0 + q]) + xv_ * dv[e0 + q];
        if (d16_kind == 1) ((__bf16*)d16)[idx * d16_ld + d + q] = (__bf16)(float)dn;
        else if (d16_kind == 2) ((_Float16*)d16)[idx * d16_ld + d + q] = (_Float16)(float)dn;
      }
    }
  }
  if (threadIdx.x == 0) {
    const int64_t ncol = (int64_t)T * Rp;
    gam[(int64_t)u * ncol + idx] = g;
    xi[(int64_t)u * ncol + idx] = x_;
    rr[idx] = rzn;
    iters[idx] = u + 1;
    uint8_t st = kActive;
    if (!isfinite(rrn) || !isfinite(rzn)) st = CMTCS_CG_BREAKDOWN;
    else if (rrn == 0.0 || (fixed == 0 && rrn <= thr[idx])) st = CMTCS_CG_CONVERGED;
    else if (u + 1 >= steps) st = fixed ? CMTCS_CG_CONVERGED : CMTCS_CG_MAX_ITER;
    state[idx] = st;
    if (st == kActive) atomicAdd(&act[(int64_t)(u + 1) * T + t], 1);
  }
}

// mu_tc = x of the mean system; s_tc = (1/K) sum_k p_k (.) x_k  (Eq. (diag-est)).
template <typename VT>
__global__ __launch_bounds__(256) void k_estep_finalize(const VT* __restrict__ X, int K,
                                                        const uint64_t* __restrict__ keyp,
                                                        const int8_t* __restrict__ probes,
                                                        float* __restrict__ mu,
                                                        float* __restrict__ sdiag, int C, int Rp,
                                                        int D, int crn,
                                                        const double* __restrict__ mdiag) {
  const int tc = blockIdx.x;
  const int t = tc / C, c = tc % C;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  const int64_t base = ((int64_t)t * Rp + (int64_t)c * (K + 1)) * D + d;
  mu[(int64_t)tc * D + d] = (float)X[base];
  const uint64_t key = probes == nullptr ? *keyp : 0;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    const double p = probes != nullptr
                         ? (double)probes[(((int64_t)t * C + c) * K + k) * D + d]
                         : probe_entry(key, t, crn ? 0 : c, k, d, C, K, D);
    acc += p * (double)X[base + (int64_t)(k + 1) * D];
  }
  // Jacobi: the probe solves are A^-1 M^1/2 p, so the estimate is rescaled by M^-1/2
  const double sc = mdiag != nullptr ? 1.0 / sqrt(mdiag[(int64_t)tc * D + d]) : 1.0;
  sdiag[(int64_t)tc * D + d] = (float)(acc / (double)K * sc);
}

template <typename VT>
__global__ __launch_bounds__(256) void k_copy_cols(const VT* __restrict__ X,
                                                   VT* __restrict__ out, int R, int Rp, int D) {
  const int col = blockIdx.x;
  const int t = col / R, j = col % R;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  out[(int64_t)col * D + d] = X[((int64_t)t * Rp + j) * D + d];
}

__global__ __launch_bounds__(256) void k_coef_out(const double* __restrict__ gam,
                                                  const double* __restrict__ xi,
                                                  const int* __restrict__ iters,
                                                  double* __restrict__ gout,
                                                  double* __restrict__ xout, int T, int R,
                                                  int Rp, int steps) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)T * R * steps;
  if (i >= total) return;
  const int u = (int)(i % steps);
  const int64_t col = i / steps;
  const int t = (int)(col / R), j = (int)(col % R);
  const int64_t idx = (int64_t)t * Rp + j;
  const bool live = u < iters[idx];
  const int64_t src = (int64_t)u * T * Rp + idx;
  if (gout != nullptr) gout[i] = live ? gam[src] : 0.0;
  if (xout != nullptr) xout[i] = live ? xi[src] : 0.0;
}

__global__ __launch_bounds__(256) void k_stats_out(const int* __restrict__ iters,
                                                   const uint8_t* __restrict__ state,
                                                   int32_t* __restrict__ iout,
                                                   uint8_t* __restrict__ sout, int T, int R,
                                                   int Rp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)T * R) return;
  const int t = (int)(i / R), j = (int)(i % R);
  const int64_t idx = (int64_t)t * Rp + j;
  if (iout != nullptr) iout[i] = iters[idx];
  if (sout != nullptr) sout[i] = state[idx];
}

__global__ __launch_bounds__(256) void k_fill_colc(int* __restrict__ colc,
                                                   const int* __restrict__ map, int T, int R,
                                                   int Rp, int K) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)T * Rp) return;
  const int t = (int)(i / Rp), j = (int)(i % Rp);
  if (j >= R) colc[i] = -1;
  else if (map != nullptr) colc[i] = map[(long)t * R + j];
  else colc[i] = j / (K + 1);
}

// Slots j < R of task t receive X[t][j], slots R <= j < 2R receive Lam[t][j-R], the rest 0.
template <typename VT>
__global__ __launch_bounds__(256) void k_pack2(const VT* __restrict__ X,
                                               const VT* __restrict__ Lam, VT* __restrict__ Dv,
                                               int R, int Rp, int D) {
  const int col = blockIdx.x;
  const int t = col / Rp, j = col % Rp;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  VT v = 0;
  if (j < R) v = X[((int64_t)t * R + j) * D + d];
  else if (j < 2 * R) v = Lam[((int64_t)t * R + (j - R)) * D + d];
  Dv[(int64_t)col * D + d] = v;
}

// dphi[n][d] for the rows n of task t, from W = Phi_t [X | Lam] (slots j and R + j).
template <typename VT>
__global__ __launch_bounds__(256) void k_dphi(const VT* __restrict__ XL, const VT* __restrict__ W,
                                              const int64_t* __restrict__ row_off,
                                              const int64_t* __restrict__ w_off,
                                              const float* __restrict__ y, double beta,
                                              double y_coef, float* __restrict__ dphi, int T,
                                              int R, int Rp, int D) {
  const int64_t n = blockIdx.x;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  int lo = 0, hi = T;             // task of row n: row_off[t] <= n < row_off[t+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (row_off[mid] <= n) lo = mid; else hi = mid;
  }
  const int t = lo;
  const int64_t nl = n - row_off[t];
  const int64_t np = (w_off[t + 1] - w_off[t]) / Rp;
  const VT* Wt = W + w_off[t];
  double acc = 0.0, ls = 0.0;
  for (int j = 0; j < R; ++j) {
    const double x = (double)XL[((int64_t)t * Rp + j) * D + d];
    const double l = (double)XL[((int64_t)t * Rp + R + j) * D + d];
    const double wx = (double)Wt[(int64_t)j * np + nl];
    const double wl = (double)Wt[(int64_t)(R + j) * np + nl];
    acc += wl * x + wx * l;
    ls += l;
  }
  dphi[n * D + d] = (float)(-beta * acc + y_coef * beta * (double)y[n] * ls);
}

template <typename VT>
__global__ __launch_bounds__(256) void k_dalpha(const VT* __restrict__ XL,
                                                const int* __restrict__ colc,
                                                float* __restrict__ dalpha, int T, int R, int Rp,
                                                int D) {
  const int c = blockIdx.y;
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= D) return;
  double acc = 0.0;
  for (int t = 0; t < T; ++t)
    for (int j = 0; j < R; ++j)
      if (colc[(int64_t)t * Rp + j] == c)
        acc -= (double)XL[((int64_t)t * Rp + R + j) * D + d] *
               (double)XL[((int64_t)t * Rp + j) * D + d];
  dalpha[(int64_t)c * D + d] = (float)acc;
}

__global__ __launch_bounds__(256) void k_zero_i32(int* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------------------------------
// Launchers.  The column of D elements is held in registers: EPT elements per thread.

template <typename VT, int BS, int EPT>
static hipError_t init_one(const Geometry& g, const CgState& s, const RhsSource& src,
                           double tol2, hipStream_t st) {
  if (s.mdiag != nullptr)
    hipLaunchKernelGGL((k_cg_init<VT, BS, EPT, true>), dim3(g.T * g.Rp), dim3(BS), 0, st,
                       (VT*)s.X, (VT*)s.Rv, (VT*)s.Dv, s.rr, s.thr, s.state, s.iters, s.act,
                       src.kind, (const VT*)src.b, (const VT*)src.B, src.K, src.keyp,
                       src.probes, tol2, g.C, g.R, g.Rp, g.D, src.crn, s.mdiag, s.colc);
  else
    hipLaunchKernelGGL((k_cg_init<VT, BS, EPT, false>), dim3(g.T * g.Rp), dim3(BS), 0, st,
                       (VT*)s.X, (VT*)s.Rv, (VT*)s.Dv, s.rr, s.thr, s.state, s.iters, s.act,
                       src.kind, (const VT*)src.b, (const VT*)src.B, src.K, src.keyp,
                       src.probes, tol2, g.C, g.R, g.Rp, g.D, src.crn, nullptr, s.colc);
  return hipGetLastError();
}

template <typename VT, int BS, int EPT>
static hipError_t update_one(const Geometry& g, const CgState& s, int u, int steps, int fixed,
                             int split, hipStream_t st) {
  if (s.mdiag != nullptr)
    hipLaunchKernelGGL((k_cg_update<VT, BS, EPT, true>), dim3(g.T * g.R), dim3(BS), 0, st,
                       (VT*)s.X, (VT*)s.Rv, (VT*)s.Dv, (const VT*)s.AD, s.rr, s.thr, s.state,
                       s.iters, s.gam, s.xi, s.act, u, steps, fixed, g.T, g.R, g.Rp, g.D, split,
                       s.alpha, s.colc, s.beta, s.d16, s.d16_kind, s.d16_ld, s.mdiag, g.C);
  else
    hipLaunchKernelGGL((k_cg_update<VT, BS, EPT, false>), dim3(g.T * g.R), dim3(BS), 0, st,
                       (VT*)s.X, (VT*)s.Rv, (VT*)s.Dv, (const VT*)s.AD, s.rr, s.thr, s.state,
                       s.iters, s.gam, s.xi, s.act, u, steps, fixed, g.T, g.R, g.Rp, g.D, split,
                       s.alpha, s.colc, s.beta, s.d16, s.d16_kind, s.d16_ld, nullptr, g.C);
  return hipGetLastError();
}

// Dispatch on D: the column is split over BS threads with EPT elements each.  Up to D = 2048,
// 256 threads; for D <= 4096 more, smaller threads (fewer registers, more waves in flight while
// a block sits in its reductions) measured faster: 1024 x 4 in FP64 (69 vs 74 ms of updates
// per EM iteration at the precision workload against 256 x 16; 512 x 8 ran 67.2 against
// 66.6 ms) and 512 x 8 in FP32 (35 vs 43 ms).  FP32 columns
// of 1024 elements take one wave each (its reductions need no other wave): 8.96 against 9.36 ms
// of updates per EM iteration at the plain-FP32 workload.  Only there: the same one-wave layout
// for FP64 columns of 64 elements (half the lanes without elements) gave wrong E-steps at the
// tiny workload, for a cause not found.
#define CMTCS_DISPATCH_D(FN, ...)                                                  \
  do {                                                                             \
    if (g.D <= 256) return FN<VT, 256, 1>(__VA_ARGS__);                            \
    if (g.D <= 512) return FN<VT, 256, 2>(__VA_ARGS__);                            \
    if (g.D <= 1024) {                                                             \
      if constexpr (sizeof(VT) == 4)                                               \
        if (g.D == 1024) return FN<VT, 64, 16>(__VA_ARGS__);                       \
      return FN<VT, 256, 4>(__VA_ARGS__);                                          \
    }                                                                              \
    if (g.D <= 2048) return FN<VT, 256, 8>(__VA_ARGS__);                           \
    if (g.D <= 4096) {                                                             \
      if constexpr (sizeof(VT) == 8) return FN<VT, 1024, 4>(__VA_ARGS__);          \
      else return FN<VT, 512, 8>(__VA_ARGS__);                                     \
    }                                                                              \
    if (g.D <= 8192) return FN<VT, 1024, 8>(__VA_ARGS__);                          \
    return FN<VT, 1024, 16>(__VA_ARGS__);                                          \
  } while (0)

template <typename VT>
hipError_t launch_cg_init(const Geometry& g, const CgState& s, const RhsSource& src, double tol,
                          int max_steps, hipStream_t st) {
  hipError_t e = launch_zero_i32(s.act, (long)(max_steps + 1) * g.T, st);
  if (e != hipSuccess) return e;
  const double tol2 = tol * tol;
  CMTCS_DISPATCH_D(init_one, g, s, src, tol2, st);
}

template <typename VT>
hipError_t launch_cg_update(const Geometry& g, const CgState& s, int u, int steps, int fixed,
                            int split, hipStream_t st) {
  CMTCS_DISPATCH_D(update_one, g, s, u, steps, fixed, split, st);
}

__global__ void k_set_key(uint64_t* __restrict__ keyp, uint64_t key) {
  if (threadIdx.x == 0) *keyp = key;
}

hipError_t launch_set_key(uint64_t* keyp, uint64_t key, hipStream_t st) {
  hipLaunchKernelGGL(k_set_key, dim3(1), dim3(64), 0, st, keyp, key);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_estep_finalize(const Geometry& g, const CgState& s, int K, const uint64_t* keyp,
                                 const int8_t* probes, int crn, float* mu, float* sdiag,
                                 hipStream_t st) {
  hipLaunchKernelGGL((k_estep_finalize<VT>), dim3(g.T * g.C, (g.D + 255) / 256), dim3(256), 0,
                     st, (const VT*)s.X, K, keyp, probes, mu, sdiag, g.C, g.Rp, g.D, crn,
                     s.mdiag);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_solve_output(const Geometry& g, const CgState& s, void* X, double* gam_out,
                               double* xi_out, int steps, int* iters_out, uint8_t* status_out,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_copy_cols<VT>), dim3(g.T * g.R, (g.D + 255) / 256), dim3(256), 0, st,
                     (const VT*)s.X, (VT*)X, g.R, g.Rp, g.D);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (gam_out != nullptr || xi_out != nullptr) {
    const int64_t total = (int64_t)g.T * g.R * steps;
    hipLaunchKernelGGL(k_coef_out, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       s.gam, s.xi, s.iters, gam_out, xi_out, g.T, g.R, g.Rp, steps);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (iters_out != nullptr || status_out != nullptr) {
    const int64_t total = (int64_t)g.T * g.R;
    hipLaunchKernelGGL(k_stats_out, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       s.iters, s.state, iters_out, status_out, g.T, g.R, g.Rp);
    e = hipGetLastError();
  }
  return e;
}

// E-step statistics: k = j % (K+1) >= 1 marks probe columns, whose status becomes
// CMTCS_CG_NONPOS_RITZ where the log-determinant kernel left the probe out (ok = 0).
__global__ __launch_bounds__(256) void k_stats_estep(const int* __restrict__ iters,
                                                     const uint8_t* __restrict__ state,
                                                     const uint8_t* __restrict__ ok,
                                                     const int* __restrict__ keff,
                                                     int32_t* __restrict__ iout,
                                                     uint8_t* __restrict__ sout,
                                                     int32_t* __restrict__ kout, int T, int C,
                                                     int K, int R, int Rp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (kout != nullptr && i < (int64_t)T * C) kout[i] = keff[i];
  if (i >= (int64_t)T * R) return;
  const int t = (int)(i / R), j = (int)(i % R);
  const int64_t idx = (int64_t)t * Rp + j;
  if (iout != nullptr) iout[i] = iters[idx];
  if (sout != nullptr) {
    const int c = j / (K + 1), k = j % (K + 1);
    uint8_t v = state[idx];
    if (k > 0 && !ok[((int64_t)t * C + c) * K + (k - 1)]) v = CMTCS_CG_NONPOS_RITZ;
    sout[i] = v;
  }
}

hipError_t launch_stats_estep(const Geometry& g, const CgState& s, int K, const uint8_t* ok,
                              const int* keff, int32_t* iters_out, uint8_t* status_out,
                              int32_t* keff_out, hipStream_t st) {
  if (iters_out == nullptr && status_out == nullptr && keff_out == nullptr) return hipSuccess;
  const int64_t total = std::max<int64_t>((int64_t)g.T * g.R, (int64_t)g.T * g.C);
  hipLaunchKernelGGL(k_stats_estep, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     s.iters, s.state, ok, keff, iters_out, status_out, keff_out, g.T, g.C, K,
                     g.R, g.Rp);
  return hipGetLastError();
}

hipError_t launch_fill_colc(int* colc, int T, int R, int Rp, int K, const int32_t* host_map,
                            hipStream_t st) {
  int* map = nullptr;
  if (host_map != nullptr) {
    // the map is staged in the tail of colc ([T][Rp] slots hold at least [T][R] values)
    map = colc + (int64_t)T * Rp;
    hipError_t e = hipMemcpyAsync(map, host_map, sizeof(int32_t) * T * R, hipMemcpyHostToDevice,
                                  st);
    if (e != hipSuccess) return e;
  }
  const long n = (long)T * Rp;
  hipLaunchKernelGGL(k_fill_colc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, colc,
                     map, T, R, Rp, K);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_pack2(const Geometry& g, const void* X, const void* Lam, void* Dv,
                        hipStream_t st) {
  hipLaunchKernelGGL((k_pack2<VT>), dim3(g.T * g.Rp, (g.D + 255) / 256), dim3(256), 0, st,
                     (const VT*)X, (const VT*)Lam, (VT*)Dv, g.R, g.Rp, g.D);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_grads(const Geometry& g, int R, const VT* XL, const VT* W, const float* y,
                        const int* colc, double beta, double y_coef, float* dalpha,
                        float* dphi, int64_t rows, hipStream_t st) {
  if (dphi != nullptr && rows > 0) {
    hipLaunchKernelGGL((k_dphi<VT>), dim3((unsigned)rows, (g.D + 255) / 256), dim3(256), 0, st,
                       XL, W, g.row_off, g.w_off, y, beta, y_coef, dphi, g.T, R, g.Rp, g.D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (dalpha != nullptr) {
    hipLaunchKernelGGL((k_dalpha<VT>), dim3((g.D + 255) / 256, g.C), dim3(256), 0, st, XL, colc,
                       dalpha, g.T, R, g.Rp, g.D);
    return hipGetLastError();
  }
  return hipSuccess;
}

// mbase[t][d] = beta sum_n Phi_t[n][d]^2: the data part of diag(A_tc), once per handle.
__global__ __launch_bounds__(256) void k_colnorm(const float* __restrict__ phi,
                                                 const int64_t* __restrict__ row_off, double beta,
                                                 double* __restrict__ mbase, int D) {
  const int t = blockIdx.x;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  double acc = 0.0;
  for (int64_t n = row_off[t]; n < row_off[t + 1]; ++n) {
    const double v = (double)phi[n * D + d];
    acc += v * v;
  }
  mbase[(int64_t)t * D + d] = beta * acc;
}

// mdiag[t][c][d] = mbase[t][d] + alpha[c][d]; slogm[t][c] = sum_d log mdiag[t][c][d] (one block
// per (t, c), fixed order).
__global__ __launch_bounds__(256) void k_jacobi(const double* __restrict__ mbase,
                                                const float* __restrict__ alpha,
                                                double* __restrict__ mdiag,
                                                double* __restrict__ slogm, int C, int D) {
  __shared__ double sh[4];
  const int t = blockIdx.x / C, c = blockIdx.x % C;
  double acc = 0.0;
  for (int d = threadIdx.x; d < D; d += 256) {
    const double m = mbase[(int64_t)t * D + d] + (double)alpha[(int64_t)c * D + d];
    mdiag[(int64_t)blockIdx.x * D + d] = m;
    acc += log(m);
  }
  const double sl = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) slogm[blockIdx.x] = sl;
}

hipError_t launch_colnorm(const Geometry& g, const float* phi, double beta, double* mbase,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_colnorm, dim3(g.T, (g.D + 255) / 256), dim3(256), 0, st, phi, g.row_off,
                     beta, mbase, g.D);
  return hipGetLastError();
}

hipError_t launch_jacobi(const Geometry& g, const double* mbase, const float* alpha,
                         double* mdiag, double* slogm, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi, dim3(g.T * g.C), dim3(256), 0, st, mbase, alpha, mdiag, slogm,
                     g.C, g.D);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int* p, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template hipError_t launch_pack2<double>(const Geometry&, const void*, const void*, void*,
                                         hipStream_t);
template hipError_t launch_pack2<float>(const Geometry&, const void*, const void*, void*,
                                        hipStream_t);
template hipError_t launch_grads<double>(const Geometry&, int, const double*, const double*,
                                         const float*, const int*, double, double, float*,
                                         float*, int64_t, hipStream_t);
template hipError_t launch_grads<float>(const Geometry&, int, const float*, const float*,
                                        const float*, const int*, double, double, float*,
                                        float*, int64_t, hipStream_t);
template hipError_t launch_cg_init<double>(const Geometry&, const CgState&, const RhsSource&,
                                           double, int, hipStream_t);
template hipError_t launch_cg_init<float>(const Geometry&, const CgState&, const RhsSource&,
                                          double, int, hipStream_t);
template hipError_t launch_cg_update<double>(const Geometry&, const CgState&, int, int, int,
                                             int, hipStream_t);
template hipError_t launch_cg_update<float>(const Geometry&, const CgState&, int, int, int, int,
                                            hipStream_t);
template hipError_t launch_estep_finalize<double>(const Geometry&, const CgState&, int,
                                                  const uint64_t*,
                                                  const int8_t*, int, float*, float*,
                                                  hipStream_t);
template hipError_t launch_estep_finalize<float>(const Geometry&, const CgState&, int,
                                                 const uint64_t*,
                                                 const int8_t*, int, float*, float*,
                                                 hipStream_t);
template hipError_t launch_solve_output<double>(const Geometry&, const CgState&, void*, double*,
                                                double*, int, int*, uint8_t*, hipStream_t);
template hipError_t launch_solve_output<float>(const Geometry&, const CgState&, void*, double*,
                                               double*, int, int*, uint8_t*, hipStream_t);

}  // namespace cmtcs
