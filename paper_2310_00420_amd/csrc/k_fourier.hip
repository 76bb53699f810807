// Partial-Fourier sensing (Sec. 4: Phi_t = Omega_t F, F the unitary D x D DFT, Omega_t a subset
// of its rows; real model through the stacking [Re; Im]), where applying A costs O(D log D)
// (Sec. 3.3):
//     A v = beta Re(F^H Omega^T Omega F v) + alpha (.) v = beta F^H diag(h) F v + alpha (.) v,
// with h_k = (m_k + m_{-k}) / 2 and m_k the number of times frequency k is selected: for a real
// v the real part averages each frequency with its mirror image, so A maps real vectors to real
// vectors through one complex transform pair with a real, symmetric multiplier.
//
// The whole CG solve of a right-hand side (Alg. 1) runs in one workgroup: the column lives in
// registers, the transforms in LDS (two buffers, so that each stage needs one barrier), and
// nothing but the step sizes gamma_u, xi_u (for the
// log-determinant, Eq. (tridiag)) and the final solution goes to HBM.  A workgroup solves two
// columns of the same task at once: since h is real and symmetric, F^H diag(h) F applied to
// v1 + i v2 gives the two real results as the real and imaginary parts, so one complex FFT pair
// serves both.  The transform is the Stockham autosort FFT (radix 8, with one radix-2 or
// radix-4 stage for the remaining factor), out of place between the two LDS buffers.
// Twiddles come from per-stage tables built by each workgroup in LDS.
#include <algorithm>

#include "internal.h"
#include "../../include/cmtcs.h"

namespace cmtcs {

namespace {

// Stages of the length-2^LOGN transform: one radix-2 or radix-4 stage for the factor that
// radix 8 leaves, then radix 8.  Stage s (sub-transform length Ns before it, radix R) uses the
// twiddles w^k = exp(-2 pi i k / (R Ns)), k < Ns, stored contiguously per stage, so that the
// lanes of a butterfly row read consecutive entries; each stage's table starts on a multiple of
// 16 entries (256 bytes), so that 16 consecutive entries fill one aligned 256-byte block.
template <int LOGN>
constexpr int first_radix() { return LOGN % 3 == 1 ? 2 : LOGN % 3 == 2 ? 4 : 8; }
constexpr int twiddle_stride(int ns) { return (ns + 15) & ~15; }
template <int LOGN>
constexpr int twiddle_len() {
  int n = 0;
  for (int ns = 1, r = first_radix<LOGN>(); ns < (1 << LOGN); ns *= r, r = 8)
    n += twiddle_stride(ns);
  return n;
}

// LDS slot of point i in a transform buffer (16 bytes per slot): bits 0-2 of i XORed with bits
// 3-5.  The slot stays in i's block of 16 (one aligned 256-byte block), so 16 lanes reading 16
// consecutive points from a multiple of 16 read one aligned block, which is conflict-free on
// gfx950; and 8 lanes storing points that differ in bits 0-2 with equal bits 3-5, or in bits
// 3-5 with equal bits 0-2 (every stage's stores are one of the two), hit 8 different 16-byte
// slots of a 128-byte bank row, also conflict-free.  For a multiple m of 64,
// swz(i + m) = swz(i) + m.
__device__ inline int swz(int i) { return i ^ ((i >> 3) & 7); }

__device__ inline d2 cmul(d2 a, d2 b) {
  return d2{__builtin_fma(a[0], b[0], -a[1] * b[1]), __builtin_fma(a[0], b[1], a[1] * b[0])};
}

// Four-point DFT (forward: exp(-2 pi i k d / 4); inverse: conjugate).
template <bool INV>
__device__ inline void dft4(d2 x0, d2 x1, d2 x2, d2 x3, d2& u0, d2& u1, d2& u2, d2& u3) {
  const d2 a0 = x0 + x2, a1 = x0 - x2, a2 = x1 + x3, a3 = x1 - x3;
  // -i a3 (forward) or +i a3 (inverse)
  const d2 ma3 = INV ? d2{-a3[1], a3[0]} : d2{a3[1], -a3[0]};
  u0 = a0 + a2;
  u1 = a1 + ma3;
  u2 = a0 - a2;
  u3 = a1 - ma3;
}

// Block sums of (a, b), every thread receiving both.  One barrier: `sh` (2 BS/64 doubles) must
// not be read by any thread any more, which holds when calls alternate between two areas (a
// thread reads the partials of call n before it reaches the barrier of call n + 1).
template <int BS>
__device__ inline d2 block_sum2_alt(double a, double b, double* sh) {
  a = wave_sum_to_63(a);
  b = wave_sum_to_63(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) { sh[2 * w] = a; sh[2 * w + 1] = b; }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) { sa += sh[2 * i]; sb += sh[2 * i + 1]; }
  return d2{sa, sb};
}

// One Stockham stage of radix R (2, 4 or 8) over N points, out of place: butterfly j
// (0 <= j < N/R) reads src[j + r N/R], multiplies input r by the twiddle w^(r k) (k = j mod Ns,
// w = exp(-2 pi i / (R Ns))), transforms the R values and writes them to
// dst[(j / Ns) R Ns + k + r Ns].  Ns is the length of the sub-transforms already done.  Every
// thread of the block must call it; one barrier at the end publishes dst.
// With one butterfly per thread (N = R BS), butterfly j = threadIdx.x reads points j + r BS and,
// when Ns = N / R, writes points j + r BS: the thread's own points in the natural order.  Then
// IN_REGS takes the inputs from vin[r] instead of src, SCALE multiplies output r by hscale
// times the r-th byte of hc (the multiplier count of point j + r BS), and OUT_REGS leaves the
// outputs in vout[r] instead of storing them (no barrier then: nothing was written).
template <int R, bool INV, int BS, int N, bool IN_REGS = false, bool SCALE = false,
          bool OUT_REGS = false>
__device__ inline void fft_stage(const d2* src, d2* dst, const d2* tw, int Ns,
                                 const d2* vin = nullptr, const uint32_t* hc = nullptr,
                                 double hscale = 0.0, d2* vout = nullptr) {
  constexpr int NBF = N / R;                       // butterflies
  constexpr int PER = NBF >= BS ? NBF / BS : 1;    // per thread
  static_assert(!(IN_REGS || SCALE || OUT_REGS) || NBF == BS,
                "own points need one butterfly per thread");
  // one butterfly at a time: their registers would otherwise crowd out the columns' state
#pragma unroll 1
  for (int i = 0; i < PER; ++i) {
    const int j = (int)threadIdx.x + i * BS;
    if (j < NBF) {
      d2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (IN_REGS) v[r] = vin[r];
        else v[r] = src[NBF % 64 == 0 ? swz(j) + r * NBF : swz(j + r * NBF)];
      }
      const int k = j & (Ns - 1);
      // w^k from the stage's table (conjugated for the inverse); its higher powers by FP64
      // complex products instead of more LDS reads.  The first stage (Ns = 1) has only w^0 = 1
      // and skips them (its calls pass Ns = 1 as a constant).
      if (Ns > 1) {
        const d2 t1 = tw[k];
        const d2 w1 = INV ? d2{t1[0], -t1[1]} : t1;
        v[1] = cmul(v[1], w1);
        if constexpr (R >= 4) {
          const d2 w2 = cmul(w1, w1), w3 = cmul(w1, w2);
          v[2] = cmul(v[2], w2);
          v[3] = cmul(v[3], w3);
          if constexpr (R == 8) {
            const d2 w4 = cmul(w2, w2);
            v[4] = cmul(v[4], w4);
            v[5] = cmul(v[5], cmul(w1, w4));
            v[6] = cmul(v[6], cmul(w2, w4));
            v[7] = cmul(v[7], cmul(w3, w4));
          }
        }
      }
      d2 u[R];
      if constexpr (R == 2) {
        u[0] = v[0] + v[1];
        u[1] = v[0] - v[1];
      } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3], u[0], u[1], u[2], u[3]);
      } else {
        // eight points: four-point transforms of the even and odd inputs, combined with the
        // eighth roots of unity exp(-+ i pi k / 4)
        d2 a[4], b[4];
        dft4<INV>(v[0], v[2], v[4], v[6], a[0], a[1], a[2], a[3]);
        dft4<INV>(v[1], v[3], v[5], v[7], b[0], b[1], b[2], b[3]);
        constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
        const d2 t1 = INV ? d2{h * (b[1][0] - b[1][1]), h * (b[1][0] + b[1][1])}
                          : d2{h * (b[1][0] + b[1][1]), h * (b[1][1] - b[1][0])};
        const d2 t2 = INV ? d2{-b[2][1], b[2][0]} : d2{b[2][1], -b[2][0]};
        const d2 t3 = INV ? d2{-h * (b[3][0] + b[3][1]), h * (b[3][0] - b[3][1])}
                          : d2{h * (b[3][1] - b[3][0]), -h * (b[3][0] + b[3][1])};
        u[0] = a[0] + b[0]; u[4] = a[0] - b[0];
        u[1] = a[1] + t1;   u[5] = a[1] - t1;
        u[2] = a[2] + t2;   u[6] = a[2] - t2;
        u[3] = a[3] + t3;   u[7] = a[3] - t3;
      }
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (SCALE) u[r] = u[r] * (hscale * (double)((hc[r / 4] >> (8 * (r % 4))) & 255u));
        if constexpr (OUT_REGS) vout[r] = u[r];
        else dst[swz(base + r * Ns)] = u[r];
      }
    }
  }
  if constexpr (!OUT_REGS) __syncthreads();
}

// Unnormalised DFT of the N points in *in (forward: exp(-2 pi i k d / N); inverse: conjugate),
// ping-ponging between the two buffers; on return *in points to the buffer holding the result.
template <bool INV, int BS, int LOGN>
__device__ inline void fft(d2** in, d2** other, const d2* tw) {
  constexpr int N = 1 << LOGN;
  int Ns = 1;
  // radix 8 where it divides, one radix-2 or radix-4 stage first for the remaining factor
  if constexpr (first_radix<LOGN>() != 8) {
    fft_stage<first_radix<LOGN>(), INV, BS, N>(*in, *other, tw, Ns);
    d2* tmp = *in; *in = *other; *other = tmp;
    tw += twiddle_stride(1);
    Ns = first_radix<LOGN>();
  }
  // a runtime loop over the radix-8 stages: unrolled, the address arithmetic of every stage is
  // invariant across CG steps and would be kept in registers
#pragma unroll 1
  for (; Ns < N; Ns *= 8) {
    fft_stage<8, INV, BS, N>(*in, *other, tw, Ns);
    d2* tmp = *in; *in = *other; *other = tmp;
    tw += twiddle_stride(Ns);
  }
}

}  // namespace

// Threads per workgroup for length 2^LOGN: a quarter of the length (four elements of each
// column in registers), at most 512 (one radix-8 butterfly per thread and stage at D = 4096),
// at least one wave.
template <int LOGN>
constexpr int fourier_bs() {
  return std::max(64, std::min(512, (1 << LOGN) / 4));
}

// Workgroup (t, pair p): columns j = 2p and 2p + 1 of task t.
//   mode 0: CG (Alg. 1) from x = 0 on the right-hand sides (kind 0: the E-step's mean system and
//           probes; kind 1: B), recording gamma_u, xi_u, the step count and the outcome, and
//           writing x to X;
//   mode 1: one application of A to B's columns, written to X.
template <int LOGN>
__global__ __launch_bounds__(fourier_bs<LOGN>()) void k_fourier_cg(
    double* __restrict__ X, double* __restrict__ gam, double* __restrict__ xi,
    int* __restrict__ iters, uint8_t* __restrict__ state, const int* __restrict__ hcount,
    const float* __restrict__ alpha, const int* __restrict__ colc, int mode, int kind,
    const double* __restrict__ b, const double* __restrict__ B, int K,
    const uint64_t* __restrict__ keyp, const int8_t* __restrict__ probes, int crn, double beta,
    double tol2, int steps, int fixed, int T, int C, int R, int Rp) {
  constexpr int N = 1 << LOGN, BS = fourier_bs<LOGN>(), E = N / BS;

  extern __shared__ double lds[];
  d2* bufA = reinterpret_cast<d2*>(lds);           // two buffers of N complex points
  d2* bufB = bufA + N;
  d2* tw = bufB + N;                               // twiddles of every stage
  // partial sums: two areas of 2 BS/64 doubles, alternated by successive reductions
  double* red = reinterpret_cast<double*>(tw + twiddle_len<LOGN>());
  double* red2 = red + 2 * (BS / 64);
  const int tid = threadIdx.x;
  // LDS slot of the thread's point e: swz(tid + e BS) = swz(tid) + e BS
  static_assert(BS % 64 == 0, "whole waves");
  const int ptid = swz(tid);
  const int pairs = Rp / 2;
  const int t = blockIdx.x / pairs, p = blockIdx.x % pairs;
  const int j0 = 2 * p;
  {
    int off = 0;
    for (int ns = 1, r = first_radix<LOGN>(); ns < N; ns *= r, r = 8) {
      for (int k = tid; k < ns; k += BS) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)(r * ns), &sn, &cs);
        tw[off + k] = d2{cs, -sn};
      }
      off += twiddle_stride(ns);
    }
  }

  // the two columns: right-hand sides, diagonal terms, multipliers
  // x, r and d of both columns stay in registers, and so do alpha of each column's cluster
  // (float) and the multiplier counts of the thread's frequencies (one byte each)
  double xv[2][E], rv[2][E], dv[2][E];
  float al[2][E];
  uint32_t hcp[(E + 3) / 4];
  bool live[2];
  uint64_t key = 0;
  if (kind == 0 && probes == nullptr) key = *keyp;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int j = j0 + q;
    live[q] = j < R;
    const int64_t idx = (int64_t)t * Rp + j;
    const int c = live[q] ? colc[idx] : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int d = tid + e * BS;
      double v = 0.0;
      if (live[q]) {
        if (kind == 0) {
          const int cc = j / (K + 1), k = j % (K + 1);
          if (k == 0) v = b[(int64_t)t * N + d];
          else if (probes != nullptr)
            v = (double)probes[(((int64_t)t * C + cc) * K + (k - 1)) * N + d];
          else v = probe_entry(key, t, crn ? 0 : cc, k - 1, d, C, K, N);
        } else {
          v = B[((int64_t)t * R + j) * N + d];
        }
      }
      xv[q][e] = 0.0;
      rv[q][e] = v;
      dv[q][e] = v;
      al[q][e] = live[q] ? alpha[(int64_t)c * N + d] : 0.0f;
    }
  }
  const double hscale = 0.5 * beta / (double)N;   // h = count / 2, beta, the pair's 1/N
#pragma unroll
  for (int i = 0; i < (E + 3) / 4; ++i) hcp[i] = 0;
#pragma unroll
  for (int e = 0; e < E; ++e)
    hcp[e / 4] |= (uint32_t)min(hcount[(int64_t)t * N + tid + e * BS], 255) << (8 * (e % 4));

  // beta Phi^T Phi d for both columns (zero for a stopped one), left in *res as (column 0,
  // column 1) pairs in natural order; A d = that + alpha (.) d is formed where it is read.  The
  // first write goes to bufA: every thread has finished reading the previous step's result by
  // then (two block reductions lie in between).
  const d2* res = bufA;
  // With radix 8 throughout and one butterfly per thread (D = 4096), a stage with Ns = 1 reads
  // exactly the thread's own points and one with Ns = N / 8 writes them.  So the forward
  // transform's first stage takes d from registers, and its last stage, the multiplier and the
  // inverse transform's first stage run on the same registers with no store, barrier or load in
  // between.  The same operations in the same order.
  constexpr bool kOwn = N == 8 * BS && first_radix<LOGN>() == 8;
  auto apply = [&](const bool* on) __attribute__((always_inline)) {
    d2* in = bufA;
    d2* other = bufB;
    if constexpr (kOwn) {
      d2 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = d2{on[0] ? dv[0][e] : 0.0, on[1] ? dv[1][e] : 0.0};
      // the previous step's result (bufA) was last read before the residual's block reduction
      fft_stage<8, false, BS, N, true>(nullptr, bufA, tw, 1, v);
      const d2* t = tw + twiddle_stride(1);
      int Ns = 8;
#pragma unroll 1
      for (; Ns < N / 8; Ns *= 8) {
        fft_stage<8, false, BS, N>(in, other, t, Ns);
        d2* tmp = in; in = other; other = tmp;
        t += twiddle_stride(Ns);
      }
      fft_stage<8, false, BS, N, false, true, true>(in, nullptr, t, Ns, nullptr, hcp, hscale, v);
      // other was last read by the stage before, ahead of its barrier
      fft_stage<8, true, BS, N, true>(nullptr, other, tw, 1, v);
      { d2* tmp = in; in = other; other = tmp; }
      t = tw + twiddle_stride(1);
#pragma unroll 1
      for (Ns = 8; Ns < N; Ns *= 8) {
        fft_stage<8, true, BS, N>(in, other, t, Ns);
        d2* tmp = in; in = other; other = tmp;
        t += twiddle_stride(Ns);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e)
        bufA[ptid + e * BS] = d2{on[0] ? dv[0][e] : 0.0, on[1] ? dv[1][e] : 0.0};
      __syncthreads();
      fft<false, BS, LOGN>(&in, &other, tw);
#pragma unroll
      for (int e = 0; e < E; ++e)
        in[ptid + e * BS] =
            in[ptid + e * BS] * (hscale * (double)((hcp[e / 4] >> (8 * (e % 4))) & 255u));
      __syncthreads();
      fft<true, BS, LOGN>(&in, &other, tw);
    }
    res = in;
  };
  auto ad_of = [&](int q, int e) __attribute__((always_inline)) {
    return __builtin_fma((double)al[q][e], dv[q][e], res[ptid + e * BS][q]);
  };

  if (mode == 1) {
    __syncthreads();   // the twiddle tables
    apply(live);
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (live[q]) {
        const int64_t base = ((int64_t)t * Rp + j0 + q) * N;
#pragma unroll
        for (int e = 0; e < E; ++e) X[base + tid + e * BS] = ad_of(q, e);
      }
    return;
  }

  double pr0 = 0.0, pr1 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    pr0 += rv[0][e] * rv[0][e];
    pr1 += rv[1][e] * rv[1][e];
  }
  const d2 r0 = block_sum2_alt<BS>(pr0, pr1, red);   // its barrier also publishes the table
  double rr[2] = {r0[0], r0[1]}, thr[2];
  bool act[2];
  uint8_t st[2];
  int its[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    thr[q] = tol2 * rr[q];
    if (!isfinite(rr[q])) st[q] = CMTCS_CG_BREAKDOWN;
    else if (rr[q] > 0.0) st[q] = kActive;
    else st[q] = CMTCS_CG_CONVERGED;   // b = 0: x = 0 is exact
    act[q] = live[q] && st[q] == kActive;
  }
  const int64_t ncol = (int64_t)T * Rp;
  for (int u = 0; u < steps && (act[0] || act[1]); ++u) {
    apply(act);
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      p0 += dv[0][e] * ad_of(0, e);
      p1 += dv[1][e] * ad_of(1, e);
    }
    const d2 dAd = block_sum2_alt<BS>(p0, p1, red2);
    double g[2] = {0.0, 0.0};
    bool upd[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      upd[q] = act[q];
      if (act[q] && (!(dAd[q] > 0.0) || !isfinite(dAd[q]))) {
        st[q] = CMTCS_CG_BREAKDOWN;   // stop before this step
        act[q] = false;
        upd[q] = false;
      }
      if (upd[q]) g[q] = rr[q] / dAd[q];
    }
    p0 = 0.0;
    p1 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (upd[q]) {
          xv[q][e] = __builtin_fma(g[q], dv[q][e], xv[q][e]);
          rv[q][e] = __builtin_fma(-g[q], ad_of(q, e), rv[q][e]);
        }
      p0 += rv[0][e] * rv[0][e];
      p1 += rv[1][e] * rv[1][e];
    }
    const d2 rrn = block_sum2_alt<BS>(p0, p1, red);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!upd[q]) continue;
      const double x_ = rrn[q] / rr[q];
#pragma unroll
      for (int e = 0; e < E; ++e) dv[q][e] = __builtin_fma(x_, dv[q][e], rv[q][e]);
      const int64_t idx = (int64_t)t * Rp + j0 + q;
      if (tid == 0) {
        gam[(int64_t)u * ncol + idx] = g[q];
        xi[(int64_t)u * ncol + idx] = x_;
      }
      rr[q] = rrn[q];
      its[q] = u + 1;
      if (!isfinite(rrn[q])) st[q] = CMTCS_CG_BREAKDOWN;
      else if (rrn[q] == 0.0 || (fixed == 0 && rrn[q] <= thr[q])) st[q] = CMTCS_CG_CONVERGED;
      else if (u + 1 >= steps) st[q] = fixed ? CMTCS_CG_CONVERGED : CMTCS_CG_MAX_ITER;
      act[q] = st[q] == kActive;
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (!live[q]) continue;
    const int64_t idx = (int64_t)t * Rp + j0 + q;
    const int64_t base = idx * N;
#pragma unroll
    for (int e = 0; e < E; ++e) X[base + tid + e * BS] = xv[q][e];
    if (tid == 0) {
      iters[idx] = its[q];
      // a column still active here ran out of steps (steps = 0)
      state[idx] = st[q] == kActive ? (fixed ? CMTCS_CG_CONVERGED : CMTCS_CG_MAX_ITER) : st[q];
    }
  }
}

// b_t[d] = beta Re(F^H Omega_t^T y_t)[d] = beta / sqrt(D) sum_n (Re y_n cos(2 pi k_n d / D)
//          - Im y_n sin(2 pi k_n d / D)), the angle reduced exactly: (k_n d) mod D.
__global__ __launch_bounds__(256) void k_fourier_rhs(const int* __restrict__ freq,
                                                     const float* __restrict__ yc,
                                                     const int64_t* __restrict__ row_off,
                                                     double beta, double* __restrict__ b,
                                                     int D) {
  const int t = blockIdx.x;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  double acc = 0.0;
  for (int64_t n = row_off[t]; n < row_off[t + 1]; ++n) {
    const int k = freq[n];
    if (k < 0 || k >= D) continue;   // rejected at create
    const int64_t m = ((int64_t)k * d) & (D - 1);
    double sn, cs;
    sincospi(2.0 * (double)m / (double)D, &sn, &cs);
    acc += (double)yc[2 * n] * cs - (double)yc[2 * n + 1] * sn;
  }
  b[(int64_t)t * D + d] = beta * acc / sqrt((double)D);
}

// hcount[t][k] = m_k + m_{-k}: selections of frequency k and of its mirror (D - k) mod D.
// Frequencies outside [0, D) are counted in *bad and otherwise ignored.
__global__ __launch_bounds__(256) void k_fourier_hcount(const int* __restrict__ freq,
                                                        const int64_t* __restrict__ row_off,
                                                        int* __restrict__ hcount,
                                                        int* __restrict__ bad, int T, int D) {
  const int t = blockIdx.x;
  for (int64_t n = row_off[t] + threadIdx.x; n < row_off[t + 1]; n += 256) {
    const int k = freq[n];
    if (k < 0 || k >= D) {
      atomicAdd(bad, 1);
      continue;
    }
    atomicAdd(&hcount[(int64_t)t * D + k], 1);
    atomicAdd(&hcount[(int64_t)t * D + ((D - k) & (D - 1))], 1);
  }
}

template <int LOGN>
static hipError_t fourier_one(const Geometry& g, const CgState& s, const int* hcount, int mode,
                              const RhsSource& src, double tol2, int steps, int fixed,
                              hipStream_t st) {
  constexpr int N = 1 << LOGN, BS = fourier_bs<LOGN>();
  // two buffers of N complex points, the twiddle tables, the reduction slots
  const size_t lds =
      sizeof(double) * (4 * N + 2 * twiddle_len<LOGN>() + 4 * (BS / 64));
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fourier_cg<LOGN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_fourier_cg<LOGN>, dim3((unsigned)(g.T * (g.Rp / 2))), dim3(BS), lds, st,
                     (double*)s.X, s.gam, s.xi, s.iters, s.state, hcount, s.alpha, s.colc, mode,
                     src.kind, (const double*)src.b, (const double*)src.B, src.K, src.keyp,
                     src.probes, src.crn, s.beta, tol2, steps, fixed, g.T, g.C, g.R, g.Rp);
  return hipGetLastError();
}

hipError_t launch_fourier_cg(const Geometry& g, const CgState& s, const int* hcount, int mode,
                             const RhsSource& src, double tol, int steps, int fixed,
                             hipStream_t st) {
  const double tol2 = tol * tol;
  switch (g.D) {
    case 64: return fourier_one<6>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 128: return fourier_one<7>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 256: return fourier_one<8>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 512: return fourier_one<9>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 1024: return fourier_one<10>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 2048: return fourier_one<11>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    case 4096: return fourier_one<12>(g, s, hcount, mode, src, tol2, steps, fixed, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fourier_setup(const Geometry& g, const int* freq, const float* yc, double beta,
                                double* b, int* hcount, int* bad, hipStream_t st) {
  hipError_t e = hipMemsetAsync(hcount, 0, sizeof(int) * (size_t)g.T * g.D, st);
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fourier_hcount, dim3(g.T), dim3(256), 0, st, freq, g.row_off, hcount, bad,
                     g.T, g.D);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fourier_rhs, dim3(g.T, (g.D + 255) / 256), dim3(256), 0, st, freq, yc,
                     g.row_off, beta, b, g.D);
  return hipGetLastError();
}

}  // namespace cmtcs
