// Mixed-precision operator (CMTCS_MATH_MIXED): Phi stored in 16 bits (bf16 or fp16), the CG
// direction rounded to the same type, products on the 16x16x32 matrix cores with FP32
// accumulation (the precision form of the solver; the method itself is Alg. 1 on the operator of
// Eq. (lin-sys)).
//
// Both products are laid out so that the contraction index is contiguous in memory for both
// operands (one 16-byte load gives a lane its 8 consecutive k values):
//   fwd:  W16_t = round16(Phi16_t V16_t)       M = Phi16_t   [N_t][D]   (caller's rows), K = D
//   adj:  AV_t  = beta PhiT16_t W16_t + alpha (.) V_t
//                                              M = PhiT16_t  [D][np_t] (built once at create,
//                                              a transposed copy: HBM is plentiful, and the
//                                              16-bit path is bound by streaming Phi)
// np_t = N_t rounded up to 32; W16_t is [Rp][np_t] with zero rows beyond N_t.  Every 16-bit
// array has the padded row pitch ld16 (Phi16 and the direction ld16(D), PhiT16 and W16
// ld16(np_t)); the padding is never read.
// The true residual b - A x that replaces the recursive residual every m steps is computed by
// the FP32 kernels of k_operator.hip from the FP32 copy of Phi.
#include <type_traits>

#include "internal.h"
#include "../../include/cmtcs.h"

namespace cmtcs {

template <typename T16> struct Mfma16;
template <> struct Mfma16<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  __device__ static inline f4 mma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  __device__ static inline f4 mma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__device__ inline int xcd_block16(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, rem) + i;
}

constexpr int kRF16 = kRows16 / 16;   // 64 output rows per wave tile

// Shared main loop: acc[rf][cf] += M[rows of rf][k] * V[cols of cf][k] over k in [0, K), K a
// multiple of 32.  mrow[rf] points at row (tile row rf*16 + i16) + 8*g4 (a row past the end of
// M points at a valid row instead, and the caller drops its outputs); vcol points at column
// (cf0*16 + i16) + 8*g4, columns vld elements apart.  As in the FP64/FP32 products, every load
// is unconditional (chunk index clamped, a missing column fragment re-reads the last present
// one) and no loaded value is touched before its MFMA, so each chunk waits only for the buffer
// it multiplies.
// Shared main loop of the 16-bit products for one block of four waves (four consecutive 64-row
// tiles of one task and column group): acc[rf][cf] += M[rows of rf][k] * V[cols of cf][k] over
// k in [0, K), K a multiple of 32.  mrow[rf] points at this wave's row (tile row rf*16 + i16)
// + 8*g4 (a row past the end of M points at a valid row, whose outputs the caller drops); vsrc
// points at column cf0*16 of the right-hand-side block, columns vld elements apart.
//
// The right-hand-side chunk (32 k x up to 144 columns, 9 KB) that all four waves multiply is
// staged once per block into an LDS double buffer (rows padded to 80 bytes, so that the eight
// lanes served together read distinct banks): loading it per wave made the kernel bound by the
// CU's vector-memory throughput.  Phi is prefetched kRing16 - 1 chunks ahead in registers.  As in
// the FP64/FP32 products, every load is unconditional, and the first round is peeled so that
// the accumulators start in the matrix-core result registers.
constexpr int kRing16 = 4;
constexpr int kStg16 = 2;   // staged chunks in flight in registers (divides kRing16)
constexpr int kLd16 = 40;                                      // padded LDS row (elements)
constexpr int kPieces16 = 4;                                   // 16-byte pieces per column chunk
constexpr int kPer16 = (16 * kColGroup * kPieces16 + 255) / 256;

template <typename T16>
__device__ inline void nt16_mainloop(f4 (&acc)[kRF16][kColGroup], const T16* const (&mrow)[kRF16],
                                     const T16* vsrc, int64_t vld, int ncf, int K,
                                     T16 (*lds)[16 * kColGroup][kLd16]) {
  typedef typename Mfma16<T16>::v8 v8;
  const int lane = threadIdx.x & 63, i16 = lane & 15, g4 = lane >> 4;
  const int nch = K / 32;
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int rf = 0; rf < kRF16; ++rf)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf) acc[rf][cf] = f4{0.f, 0.f, 0.f, 0.f};
  };
  if (nch == 0) { zero_acc(); return; }   // uniform over the block
  // staging: piece p is column p / kPieces16, 16-byte piece p % kPieces16; pieces past the
  // group's columns are clamped onto the last one (a duplicate load and an identical store)
  const int npieces = 16 * ncf * kPieces16;
  const T16* ssrc[kPer16];
  T16* sdst[2][kPer16];
#pragma unroll
  for (int i = 0; i < kPer16; ++i) {
    const int p = min((int)threadIdx.x + i * 256, npieces - 1);
    const int col = p / kPieces16, q = p % kPieces16;
    ssrc[i] = vsrc + (int64_t)col * vld + q * 8;
    sdst[0][i] = &lds[0][col][q * 8];
    sdst[1][i] = &lds[1][col][q * 8];
  }
  v8 a[kRing16][kRF16], stg[kStg16][kPer16];
  auto load_a = [&](v8 (&x)[kRF16], int c) __attribute__((always_inline)) {
    const int k0 = min(c, nch - 1) * 32;
#pragma unroll
    for (int rf = 0; rf < kRF16; ++rf) x[rf] = *(const v8*)(mrow[rf] + k0);
  };
  auto stage_load = [&](v8 (&x)[kPer16], int c) __attribute__((always_inline)) {
    const int k0 = min(c, nch - 1) * 32;
#pragma unroll
    for (int i = 0; i < kPer16; ++i) x[i] = *(const v8*)(ssrc[i] + k0);
  };
  auto stage_store = [&](const v8 (&x)[kPer16], int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < kPer16; ++i) *(v8*)sdst[buf][i] = x[i];
  };
  auto step = [&](const v8 (&x)[kRF16], int buf, auto full, auto first)
      __attribute__((always_inline)) {
    v8 bv[kColGroup];
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf)
      if (decltype(full)::value || cf < ncf) bv[cf] = *(const v8*)&lds[buf][cf * 16 + i16][8 * g4];
    // all nine reads in flight before the first product (the scheduler would otherwise pair
    // each read with its products and wait out the LDS latency nine times)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf)
      if (decltype(full)::value || cf < ncf)
#pragma unroll
        for (int rf = 0; rf < kRF16; ++rf) {
          const f4 cin = decltype(first)::value ? f4{0.f, 0.f, 0.f, 0.f} : acc[rf][cf];
          acc[rf][cf] = Mfma16<T16>::mma(x[rf], bv[cf], cin);
        }
  };
  // per chunk c (buffer c & 1): multiply; store the staged chunk c+1 into the other buffer
  // (whose chunk c-1 every wave finished before the last barrier); stage chunk c+1+kStg16 into
  // the registers just stored from; then the Phi load of chunk c + kRing16 - 1 (after the
  // staging loads: the memory counter completes in issue order); barrier.  A staged chunk is
  // loaded kStg16 chunks before it is stored, the Phi operand kRing16 - 1 before it is used.
  auto chunk = [&](int c, auto ic, auto full, auto first) __attribute__((always_inline)) {
    constexpr int i = decltype(ic)::value;
    constexpr int si = (i + 1) % kStg16;
    step(a[i], i & 1, full, first);
    stage_store(stg[si], (i + 1) & 1);
    stage_load(stg[si], c + i + 1 + kStg16);
    load_a(a[(i + kRing16 - 1) % kRing16], c + i + kRing16 - 1);
    __syncthreads();
  };
  auto ring = [&](int c, auto full, auto first) __attribute__((always_inline)) {
    static_for<kRing16>([&](auto ic) __attribute__((always_inline)) {
      chunk(c, ic, full,
            std::integral_constant<bool, decltype(first)::value && decltype(ic)::value == 0>{});
    });
  };
  auto run = [&](auto full) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < kStg16; ++i) stage_load(stg[i], i);
#pragma unroll
    for (int i = 0; i + 1 < kRing16; ++i) load_a(a[i], i);
    stage_store(stg[0], 0);
    stage_load(stg[0], kStg16);
    __syncthreads();
    int c = 0;
    if (nch >= kRing16) {   // kRing16 is even: chunk c + i is in buffer i & 1
      ring(0, full, std::true_type{});
      for (c = kRing16; c + kRing16 <= nch; c += kRing16) ring(c, full, std::false_type{});
    } else {
      zero_acc();
    }
#pragma unroll
    for (int i = 0; i + 1 < kRing16; ++i) {
      if (c + i >= nch) break;
      step(a[i], i & 1, full, std::false_type{});
      stage_store(stg[(i + 1) % kStg16], (i + 1) & 1);
      stage_load(stg[(i + 1) % kStg16], c + i + 1 + kStg16);
      __syncthreads();
    }
  };
  if (ncf == kColGroup) run(std::true_type{});
  else run(std::false_type{});
}

// W16_t = round16(Phi16_t V16_t): tile {t, n0, column group}.
template <typename T16>
__global__ __launch_bounds__(256) void k_phi_v16(const T16* __restrict__ phi16,
                                                 const int64_t* __restrict__ row_off,
                                                 const int64_t* __restrict__ w16_off,
                                                 const int4* __restrict__ tiles, int ntiles,
                                                 const T16* __restrict__ V16,
                                                 T16* __restrict__ W16,
                                                 const int* __restrict__ act, int D, int Rp) {
  __shared__ T16 lds[2][16 * kColGroup][kLd16];
  const int lane = threadIdx.x & 63, i16 = lane & 15, g4 = lane >> 4;
  // one tile per block: four waves of kRows16 rows each
  const int blk = uniform(xcd_block16(blockIdx.x, gridDim.x));
  if (blk >= ntiles) return;
  const int4 tl = tiles[blk];
  const int t = uniform(tl.x), cf0 = uniform(tl.z) * kColGroup;
  const int n0 = uniform(tl.y) + uniform((int)(threadIdx.x >> 6)) * kRows16;
  if (act != nullptr && act[t] == 0) return;   // uniform over the block
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (nt + 31) / 32 * 32;
  const int64_t ldw = (w16_off[t + 1] - w16_off[t]) / Rp, ldd = ld16(D);
  const int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  // rows past N_t read row 0 of the task; the epilogue writes their outputs as zeros
  const T16* mrow[kRF16];
#pragma unroll
  for (int rf = 0; rf < kRF16; ++rf) {
    const int row = n0 + rf * 16 + i16;
    mrow[rf] = phi16 + (r0 + (row < nt ? row : 0)) * ldd + 8 * g4;
  }
  f4 acc[kRF16][kColGroup];
  nt16_mainloop<T16>(acc, mrow, V16 + ((int64_t)t * Rp + cf0 * 16) * ldd, ldd, ncf, D, lds);
  typedef T16 t4 __attribute__((ext_vector_type(4)));
  T16* Wt = W16 + w16_off[t];
#pragma unroll
  for (int rf = 0; rf < kRF16; ++rf) {
    const int rb = n0 + rf * 16;
    if (rb >= np) continue;
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (cf >= ncf) continue;
      const int j = (cf0 + cf) * 16 + i16;
      t4 o;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = rb + 4 * g4 + r < nt ? (T16)acc[rf][cf][r] : (T16)0.f;
      *(t4*)(Wt + (int64_t)j * ldw + rb + 4 * g4) = o;
    }
  }
}

// AV_t = beta PhiT16_t W16_t + alpha_{c(j)} (.) V_t: tile {t, d0, column group}; with no alpha,
// the bare PhiT16_t W16_t (the CG update then adds beta and the diagonal term).
template <typename T16>
__global__ __launch_bounds__(256) void k_phit_w16(const T16* __restrict__ phiT16,
                                                  const int64_t* __restrict__ row_off,
                                                  const int64_t* __restrict__ w16_off,
                                                  const int4* __restrict__ tiles, int ntiles,
                                                  const T16* __restrict__ W16,
                                                  const float* __restrict__ V,
                                                  float* __restrict__ AV,
                                                  const float* __restrict__ alpha,
                                                  const int* __restrict__ colc, double beta,
                                                  const int* __restrict__ act, int D, int Rp) {
  __shared__ T16 lds[2][16 * kColGroup][kLd16];
  const int lane = threadIdx.x & 63, i16 = lane & 15, g4 = lane >> 4;
  // one tile per block: four waves of kRows16 rows (of d) each
  const int blk = uniform(xcd_block16(blockIdx.x, gridDim.x));
  if (blk >= ntiles) return;
  const int4 tl = tiles[blk];
  const int t = uniform(tl.x), cf0 = uniform(tl.z) * kColGroup;
  const int d0 = uniform(tl.y) + uniform((int)(threadIdx.x >> 6)) * kRows16;
  if (act != nullptr && act[t] == 0) return;   // uniform over the block
  const int64_t wo = w16_off[t];
  const int np = (int)((row_off[t + 1] - row_off[t] + 31) / 32 * 32);
  const int64_t ldw = (w16_off[t + 1] - wo) / Rp;
  const int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  const T16* M = phiT16 + (wo / Rp) * (int64_t)D;
  // rows past D read row 0; their outputs are not stored
  const T16* mrow[kRF16];
#pragma unroll
  for (int rf = 0; rf < kRF16; ++rf) {
    const int row = d0 + rf * 16 + i16;
    mrow[rf] = M + (int64_t)(row < D ? row : 0) * ldw + 8 * g4;
  }
  f4 acc[kRF16][kColGroup];
  nt16_mainloop<T16>(acc, mrow, W16 + wo + (int64_t)(cf0 * 16) * ldw, ldw, ncf, np, lds);
  if (alpha == nullptr) {   // bare product: stores only
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (cf >= ncf) continue;
      const int64_t col = ((int64_t)t * Rp + (cf0 + cf) * 16 + i16) * D;
#pragma unroll
      for (int rf = 0; rf < kRF16; ++rf) {
        const int d = d0 + rf * 16 + 4 * g4;
        if (d < D) *(f4*)(AV + col + d) = acc[rf][cf];
      }
    }
    return;
  }
#pragma unroll
  for (int cf = 0; cf < kColGroup; ++cf) {
    if (cf >= ncf) continue;
    const int j = (cf0 + cf) * 16 + i16;
    const int c = colc[(int64_t)t * Rp + j];
    const int64_t col = ((int64_t)t * Rp + j) * D;
    const float* al = alpha + (int64_t)(c >= 0 ? c : 0) * D;
#pragma unroll
    for (int rf = 0; rf < kRF16; ++rf) {
      const int d = d0 + rf * 16 + 4 * g4;
      if (d >= D) continue;
      const f4 v = *(const f4*)(V + col + d);
      f4 o;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        o[r] = (float)beta * acc[rf][cf][r] + (c >= 0 ? al[d + r] : 0.f) * v[r];
      *(f4*)(AV + col + d) = o;
    }
  }
}

// PhiT16 of every task: [D][np_t] (pitch ld16(np_t)) with zero columns N_t <= n < np_t.
// 32x32 tiles through LDS.
template <typename T16>
__global__ __launch_bounds__(256) void k_transpose16(const T16* __restrict__ phi16,
                                                     const int64_t* __restrict__ row_off,
                                                     const int64_t* __restrict__ w16_off,
                                                     T16* __restrict__ phiT16, int D, int Rp) {
  __shared__ T16 tileb[32][33];
  const int t = blockIdx.z;
  const int64_t wo = w16_off[t];
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (nt + 31) / 32 * 32;
  const int64_t ldw = (w16_off[t + 1] - wo) / Rp, ldd = ld16(D);
  const int n0 = blockIdx.y * 32, d0 = blockIdx.x * 32;
  if (n0 >= np) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int n = n0 + i, d = d0 + tx;
    tileb[i][tx] = (n < nt && d < D) ? phi16[(r0 + n) * ldd + d] : (T16)0.f;
  }
  __syncthreads();
  T16* out = phiT16 + (wo / Rp) * (int64_t)D;
  for (int i = ty; i < 32; i += 8) {
    const int d = d0 + i, n = n0 + tx;
    if (d < D) out[(int64_t)d * ldw + n] = tileb[tx][i];
  }
}

// y[r][c] = round16(x[r][c]); four consecutive elements of one row per thread (cols is a
// multiple of 4 where the rows' starts are 16-byte aligned; otherwise element by element).
template <typename T16>
__global__ __launch_bounds__(256) void k_round16(const float* __restrict__ x, int64_t ldx,
                                                 T16* __restrict__ y, int64_t ldy, int64_t rows,
                                                 int cols) {
  const int quads = (cols + 3) / 4;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * quads) return;
  const int64_t r = i / quads;
  const int c = (int)(i - r * quads) * 4;
  const float* xr = x + r * ldx;
  T16* yr = y + r * ldy;
  if (c + 3 < cols && (ldx & 3) == 0 && (ldy & 3) == 0) {
    const f4 v = *(const f4*)(xr + c);
    typedef T16 t4 __attribute__((ext_vector_type(4)));
    t4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (T16)v[k];
    *(t4*)(yr + c) = o;
  } else {
    for (int k = c; k < c + 4 && k < cols; ++k) yr[k] = (T16)xr[k];
  }
}

// Second half of a residual-replacement step u for every active column:
//   r = src - A x;  xi = r.r / r_old.r_old;  d = r + xi d;  stop decision as in k_cg_update.
template <int BS, int EPT>
__global__ __launch_bounds__(BS) void k_replace(const float* __restrict__ AX,
                                                float* __restrict__ Rv, float* __restrict__ Dv,
                                                double* __restrict__ rr,
                                                const double* __restrict__ thr,
                                                uint8_t* __restrict__ state,
                                                int* __restrict__ iters,
                                                double* __restrict__ xi, int* __restrict__ act,
                                                int kind, const float* __restrict__ b,
                                                const float* __restrict__ B, int K,
                                                const uint64_t* __restrict__ keyp,
                                                const int8_t* __restrict__ probes, int u,
                                                int steps, int fixed, int T, int C, int R,
                                                int Rp, int D, int crn) {
  __shared__ double sh[BS / 64];
  const int t = blockIdx.x / R, j = blockIdx.x % R;
  const int64_t idx = (int64_t)t * Rp + j;
  if (state[idx] != kActive) return;
  const double rr_old = rr[idx];
  int c = 0, k = 0;
  uint64_t key = 0;
  if (kind == 0) {
    c = j / (K + 1);
    k = j % (K + 1);
    if (probes == nullptr) key = *keyp;
  }
  const int64_t base = idx * D;
  float rv[EPT];
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int d = threadIdx.x + e * BS;
    rv[e] = 0.f;
    if (d >= D) continue;
    float v;
    if (kind == 0) {
      if (k == 0) v = b[(int64_t)t * D + d];
      else if (probes != nullptr) v = (float)probes[(((int64_t)t * C + c) * K + (k - 1)) * D + d];
      else v = (float)probe_entry(key, t, crn ? 0 : c, k - 1, d, C, K, D);
    } else {
      v = B[((int64_t)t * R + j) * D + d];
    }
    rv[e] = v - AX[base + d];
    acc += (double)rv[e] * (double)rv[e];
  }
  const double rrn = block_sum<BS>(acc, sh);
  const double x_ = rrn / rr_old;
  const float xf = (float)x_;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int d = threadIdx.x + e * BS;
    if (d < D) {
      Rv[base + d] = rv[e];
      Dv[base + d] = rv[e] + xf * Dv[base + d];
    }
  }
  if (threadIdx.x == 0) {
    xi[(int64_t)u * T * Rp + idx] = x_;
    rr[idx] = rrn;
    iters[idx] = u + 1;
    uint8_t st = kActive;
    if (!isfinite(rrn)) st = CMTCS_CG_BREAKDOWN;
    else if (rrn == 0.0 || (fixed == 0 && rrn <= thr[idx])) st = CMTCS_CG_CONVERGED;
    else if (u + 1 >= steps) st = fixed ? CMTCS_CG_CONVERGED : CMTCS_CG_MAX_ITER;
    state[idx] = st;
    if (st == kActive) atomicAdd(&act[(int64_t)(u + 1) * T + t], 1);
  }
}

// ------------------------------------------------------------------------------------------

template <typename T16>
hipError_t launch_mixed_products(const Geometry& g16, const void* phi16, const void* phiT16,
                                 const int4* fwd, int nfwd, const int4* adj, int nadj,
                                 const void* V16, void* W16, const float* V, float* AV,
                                 const float* alpha, const int* colc, double beta,
                                 const int* act, int which, hipStream_t st) {
  if (which == 1) {
    if (nfwd == 0) return hipSuccess;
    hipLaunchKernelGGL((k_phi_v16<T16>), dim3(nfwd), dim3(256), 0, st,
                       (const T16*)phi16, g16.row_off, g16.w_off, fwd, nfwd, (const T16*)V16,
                       (T16*)W16, act, g16.D, g16.Rp);
    return hipGetLastError();
  }
  if (nadj == 0) return hipSuccess;
  hipLaunchKernelGGL((k_phit_w16<T16>), dim3(nadj), dim3(256), 0, st,
                     (const T16*)phiT16, g16.row_off, g16.w_off, adj, nadj, (const T16*)W16, V,
                     AV, alpha,
                     colc, beta, act, g16.D, g16.Rp);
  return hipGetLastError();
}

template <typename T16>
hipError_t launch_transpose16(const Geometry& g16, const void* phi16, void* phiT16,
                              int max_np, hipStream_t st) {
  if (max_np == 0) return hipSuccess;
  hipLaunchKernelGGL((k_transpose16<T16>), dim3((g16.D + 31) / 32, (max_np + 31) / 32, g16.T),
                     dim3(256), 0, st, (const T16*)phi16, g16.row_off, g16.w_off,
                     (T16*)phiT16, g16.D, g16.Rp);
  return hipGetLastError();
}

template <typename T16>
hipError_t launch_round16(const float* x, int64_t ldx, void* y, int64_t ldy, int64_t rows,
                          int cols, hipStream_t st) {
  const int64_t n = rows * ((cols + 3) / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_round16<T16>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x,
                     ldx, (T16*)y, ldy, rows, cols);
  return hipGetLastError();
}

template <int BS, int EPT>
static hipError_t replace_one(const Geometry& g, const CgState& s, const float* AX,
                              const RhsSource& src, int u, int steps, int fixed, hipStream_t st) {
  hipLaunchKernelGGL((k_replace<BS, EPT>), dim3(g.T * g.R), dim3(BS), 0, st, AX, (float*)s.Rv,
                     (float*)s.Dv, s.rr, s.thr, s.state, s.iters, s.xi, s.act, src.kind,
                     (const float*)src.b, (const float*)src.B, src.K, src.keyp, src.probes, u,
                     steps, fixed, g.T, g.C, g.R, g.Rp, g.D, src.crn);
  return hipGetLastError();
}

hipError_t launch_replace(const Geometry& g, const CgState& s, const float* AX,
                          const RhsSource& src, int u, int steps, int fixed, hipStream_t st) {
  if (g.D <= 256) return replace_one<256, 1>(g, s, AX, src, u, steps, fixed, st);
  if (g.D <= 512) return replace_one<256, 2>(g, s, AX, src, u, steps, fixed, st);
  if (g.D <= 1024) return replace_one<256, 4>(g, s, AX, src, u, steps, fixed, st);
  if (g.D <= 2048) return replace_one<256, 8>(g, s, AX, src, u, steps, fixed, st);
  if (g.D <= 4096) return replace_one<256, 16>(g, s, AX, src, u, steps, fixed, st);
  if (g.D <= 8192) return replace_one<1024, 8>(g, s, AX, src, u, steps, fixed, st);
  return replace_one<1024, 16>(g, s, AX, src, u, steps, fixed, st);
}

#define CMTCS_INST16(T16)                                                                      \
  template hipError_t launch_mixed_products<T16>(                                              \
      const Geometry&, const void*, const void*, const int4*, int, const int4*, int,            \
      const void*, void*, const float*, float*, const float*, const int*, double, const int*,  \
      int, hipStream_t);                                                                       \
  template hipError_t launch_transpose16<T16>(const Geometry&, const void*, void*, int,       \
                                              hipStream_t);                                    \
  template hipError_t launch_round16<T16>(const float*, int64_t, void*, int64_t, int64_t, int, \
                                          hipStream_t);
CMTCS_INST16(__bf16)
CMTCS_INST16(_Float16)

}  // namespace cmtcs
