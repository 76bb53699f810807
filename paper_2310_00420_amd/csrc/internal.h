// Internal declarations of the cmtcs HIP library: device helpers shared by the kernel files and
// the host-side launchers the C ABI layer (api.hip) calls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <stdint.h>

namespace cmtcs {

// ---------------------------------------------------------------------------------------------
// Vector types used for wide loads and stores.
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T, int N> struct VecOf;
template <> struct VecOf<float, 1> { typedef float type; };
template <> struct VecOf<float, 2> { typedef f2 type; };
template <> struct VecOf<float, 4> { typedef f4 type; };
template <> struct VecOf<double, 1> { typedef double type; };
template <> struct VecOf<double, 2> { typedef d2 type; };
template <> struct VecOf<double, 4> { typedef d4 type; };

// ---------------------------------------------------------------------------------------------
// 16x16x4 matrix-core tiles.  For both element types a wave computes D = A B + C with A 16x4,
// B 4x16: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator element r
// (r = 0..3) of lane l holds D[out_row(l / 16, r)][l % 16]; the FP32 and FP64 instructions
// differ here (rows 4 (l/16) + r versus l/16 + 4 r).  a_row(i) is a permutation of the 16 rows of
// A chosen so that row a_row(out_row(g, r)) = 4 g + r: a lane then holds four consecutive rows.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int g, int r) { return g + 4 * r; }
  __device__ static inline int a_row(int i) { return 4 * (i & 3) + (i >> 2); }
};
// FP64 4x4x4 product in four blocks: A and B take the lanes of the 16x16x4 product (block b
// holds matrix rows 4b .. 4b+3 and the same four columns), so with B's lane i16 reading column
// i16 & 3 the four blocks give 16 rows x 4 columns; lane (i16, g4) receives matrix row
// narrow_row(i16, g4), column i16 & 3.  Defined for FP64 only.
template <typename VT> __device__ VT mma4(VT a, VT b, VT c);
template <> __device__ inline double mma4<double>(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
__device__ inline int narrow_row(int i16, int g) { return g + 4 * (i16 >> 2); }
template <> struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int g, int r) { return 4 * g + r; }
  __device__ static inline int a_row(int i) { return i; }
};

// ---------------------------------------------------------------------------------------------
// Counter-based Rademacher probes (SplitMix64 finaliser; Steele, Lea & Flood 2014).
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Key of the probe stream of one EM iteration.
__host__ __device__ inline uint64_t probe_key(uint64_t seed, uint64_t em_iter) {
  return sm64_mix(seed + (em_iter + 1ull) * kGolden);
}

// Entry d of probe k of pair (t, c): +1 or -1.
__device__ inline double probe_entry(uint64_t key, int t, int c, int k, int d, int C, int K,
                                     int D) {
  const uint64_t words = (uint64_t)((D + 63) >> 6);
  const uint64_t i = (((uint64_t)t * C + c) * K + k) * words + (uint64_t)(d >> 6);
  const uint64_t w = sm64_mix(key + (i + 1ull) * kGolden);
  return ((w >> (d & 63)) & 1ull) ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------------------------
// v taken from another lane by the DPP control CTRL (row_mask, bank_mask as in the
// instruction); lanes the control leaves without a source, or outside row_mask, get 0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ inline double dpp_take(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, BANK_MASK, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, BANK_MASK, false));
}

// Sum of v over the wave, left in lane 63 (other lanes hold partial sums), through the
// register crossbar only: pairs and quads (quad permutations), the four quads of a row (row
// rotations by 4 and 8), then row 0 into row 1 and row 2 into row 3 (broadcast of lane 15)
// and rows 0-1 into rows 2-3 (broadcast of lane 31).  A fixed order of additions.
__device__ inline double wave_sum_to_63(double v) {
  v += dpp_take<0xB1>(v);          // quad_perm [1, 0, 3, 2]
  v += dpp_take<0x4E>(v);          // quad_perm [2, 3, 0, 1]
  v += dpp_take<0x124>(v);         // row_ror:4
  v += dpp_take<0x128>(v);         // row_ror:8
  v += dpp_take<0x142, 0xa>(v);    // row_bcast:15
  v += dpp_take<0x143, 0xc>(v);    // row_bcast:31
  return v;
}

// Fixed-order block reduction of two doubles at once; every thread of the block must call it
// (with every lane active) and receives both sums.  `sh` needs 2 BS/64 doubles of shared
// memory; the first barrier lets consecutive calls share it.
template <int BS>
__device__ inline d2 block_sum2(double a, double b, double* sh) {
  a = wave_sum_to_63(a);
  b = wave_sum_to_63(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 63) { sh[2 * w] = a; sh[2 * w + 1] = b; }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) { sa += sh[2 * i]; sb += sh[2 * i + 1]; }
  return d2{sa, sb};
}

// Fixed-order block reduction of doubles (deterministic run to run).  All threads of the block
// must call it; every thread receives the sum.  `sh` needs BS/64 doubles of shared memory.
template <int BS>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum_to_63(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 63) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) s += sh[i];
  return s;
}

// Buffer resources for the operator products: loads through a 128-bit descriptor (base and
// byte length in scalar registers) with a 32-bit per-lane byte offset and a wave-uniform scalar
// offset, so a load needs no per-lane 64-bit address arithmetic, and bytes past the length read
// as zeros.  Only the per-lane offset is counted against the length here: a kernel that relies
// on the zeros rebuilds the descriptor at the wave-uniform start instead of using the scalar
// offset.
// The base and length must be wave-uniform; they are moved to scalar registers explicitly
// (the compiler cannot always prove them uniform and would otherwise loop over the lanes).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ inline rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  const uint32_t n = __builtin_amdgcn_readfirstlane(bytes);
  return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0, (int)n,
                                           0x00020000);
}
template <typename T> __device__ inline T buf_load(rsrc_t r, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16 || sizeof(T) == 32,
                "load size");
  if constexpr (sizeof(T) == 32) {   // two 16-byte loads
    typedef uint32_t u8v __attribute__((ext_vector_type(8)));
    const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0);
    return __builtin_bit_cast(T, u8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
  } else if constexpr (sizeof(T) == 16)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  else if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Calls f(std::integral_constant<int, i>{}) for i = 0 .. N-1 (a compile-time unrolled loop).
template <typename F, int... I>
__device__ inline __attribute__((always_inline)) void static_for_impl(
    F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline __attribute__((always_inline)) void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// A value every lane of the wave holds equally, moved to a scalar register.
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Internal state of a right-hand side during CG.
constexpr uint8_t kActive = 255;

// ---------------------------------------------------------------------------------------------
// Geometry of one batched solve: every task has Rp column slots (a multiple of 16; the first R
// are right-hand sides, the rest zero padding) and W_t = Phi_t V_t is stored [Rp][np_t] with
// np_t = N_t rounded up to 16, task t starting at element w_off[t].
struct Geometry {
  int T, C, D, R, Rp;
  const int64_t* row_off;   // device [T+1]
  const int64_t* w_off;     // device [T+1]
  // waves of a block that split the contraction of the FP32 forward product (fwd_split_of)
  int fwd_split = 1;
  // Phi transposed per task (launch_transpose_phi) for the FP64 LDS-staged adjoint product, or
  // null (that product then reads Phi itself)
  const float* phiT = nullptr;
};

// Wave tiles of the two operator products, one int4 per tile:
//   fwd  (W = Phi V):             {t, n0, column group, 0}
//   adj  (A V = beta Phi^T W + alpha V): {t, d0, column group, 0}
// A column group is up to kColGroup 16-column fragments (144 columns) held by one wave.  All
// groups of a launch have the same width: with at most kColGroup fragments there is one group
// of all of them; beyond that the column slots are padded to a multiple of kColGroup
// fragments (zero columns), so that the products run one guard-free instantiation.
constexpr int kColGroup = 9;
// Column slots per task (a multiple of 16) for R right-hand sides.
inline int col_slots(int R) {
  const int frags = (R + 15) / 16;
  if (frags <= kColGroup) return 16 * frags;
  return 16 * kColGroup * ((frags + kColGroup - 1) / kColGroup);
}
// 16-column fragments per column group for Rp column slots.
__host__ __device__ inline int group_width(int Rp) {
  const int frags = Rp / 16;
  return frags <= kColGroup ? frags : kColGroup;
}

// Forward products of FP32 right-hand sides split the contraction over d between the four waves
// of a block when the problem has fewer 16-row tiles (over tasks and column groups) than the
// chip has SIMDs (1024): with one wave per tile most SIMDs would idle.  The choice depends on
// the problem alone, not on the tile height the autotuner picks, so that every tile height adds
// the same partial sums in the same order.  np16: sum over tasks of ceil(N_t / 16).
inline int fwd_split_of(int64_t np16, int Rp, int D) {
  const int64_t groups = Rp / 16 / group_width(Rp);
  return np16 * groups < 1024 && D >= 256 ? 4 : 1;
}

// Launchers (k_operator.hip).  `act` is the [T] count of active right-hand sides for the
// current step (tasks with a zero count are skipped) or null.  `state` is the CG loop's [T*Rp]
// column states or null: with it both products compact each task's active columns into its
// leading fragments (W then holds the columns by compacted position, so a forward and an
// adjoint product of one step take the same `state`), without it every slot is multiplied.
// `rows` is the output rows per wave tile the tile table was built for (one of
// op_row_candidates).
// phiT <- Phi_t transposed for every task: task t at element D pt_off[t], D rows of
// np_t = pt_off[t + 1] - pt_off[t] elements (np_t >= N_t; rows n >= N_t written as zeros).
// max_np: the largest np_t.  Reads Phi once and writes phiT once.
hipError_t launch_transpose_phi(const float* phi, const int64_t* row_off, const int64_t* pt_off,
                                float* phiT, int T, int D, int max_np, hipStream_t st);
template <typename VT>
hipError_t launch_phi_v(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                        const VT* V, VT* W, const int* act, const uint8_t* state, int rows,
                        hipStream_t st);
// alpha == nullptr: AV = Phi^T W alone (beta and the diagonal term are left to the caller).
template <typename VT>
hipError_t launch_phit_w(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                         const VT* W, const VT* V, VT* AV, const float* alpha, const int* colc,
                         double beta, const int* act, const uint8_t* state, int rows,
                         hipStream_t st);
// Writes the supported tile heights of product `kind` (0: Phi V, 1: Phi^T W) for FP64 (f64)
// or FP32 right-hand sides, default first, and returns their count (at most kMaxTileCands).  A
// positive height is the output rows of a one-wave tile of the register-pipelined kernels; a
// negative one selects the LDS-staged kernels, whose tile is a block of four waves of -rows rows
// each (tile_step gives the rows a tile covers).
constexpr int kMaxTileCands = 4;
int op_row_candidates(bool f64, int kind, int* rows);
inline int tile_step(int rows) { return rows > 0 ? rows : -4 * rows; }

// Launchers (k_cg.hip).
struct CgState {
  void* X; void* Rv; void* Dv; void* AD;   // [T][Rp][D] vectors of the element type
  double* rr;        // [T*Rp] current r.r
  double* thr;       // [T*Rp] tol^2 ||b||^2
  uint8_t* state;    // [T*Rp] kActive or a CMTCS_CG_* code
  int* iters;        // [T*Rp]
  double* gam;       // [max_iters][T*Rp]
  double* xi;        // [max_iters][T*Rp]
  int* act;          // [(max_iters+1)][T] active counts per step
  // Diagonal term of the operator, applied by the CG update when alpha != nullptr: AD then
  // holds the bare product Phi^T Phi d, and the update forms beta AD + alpha_{c(j)} (.) d
  // itself (it reads d anyway).  nullptr: AD already holds A d.
  const float* alpha;   // [C][D]
  const int* colc;      // [T*Rp] cluster of each column
  double beta;
  // 16-bit copy of the direction for the mixed-precision products, written by the CG update
  // beside d (same rounding as a separate conversion pass): 0 none, 1 bf16, 2 fp16
  void* d16;
  int d16_kind;
  int64_t d16_ld;   // pitch of d16's columns (elements)
  // Jacobi preconditioner (not in the paper): M = diag(A_tc), [T][C][D] FP64, or null for plain
  // CG.  With it, rr holds r.z (z = M^-1 r), d is built from z, and the stop rule still tests
  // the unpreconditioned ||r||; probe right-hand sides are M^1/2 p.
  const double* mdiag;
};
// Source of the right-hand sides for cg_init.
struct RhsSource {
  int kind;                 // 0: estep (mean b_t and probes), 1: explicit B [T][R][D]
  const void* b;            // kind 0: [T][D] b_t of the element type
  const void* B;            // kind 1
  int K;                    // kind 0
  const uint64_t* keyp;     // kind 0: device word holding the probe key (read by the kernels,
                            // so that a recorded launch sequence can be replayed with a new key)
  const int8_t* probes;     // kind 0: optional explicit probes [T][C][K][D]
  int crn;                  // kind 0, generated probes: 1 = every cluster of a task uses the
                            // probes of cluster 0 (common random numbers)
};
template <typename VT>
hipError_t launch_cg_init(const Geometry& g, const CgState& s, const RhsSource& src,
                          double tol, int max_steps, hipStream_t st);
// split = 1: first half of a residual-replacement step (x and recursive r, gamma recorded);
// launch_replace completes it.
template <typename VT>
hipError_t launch_cg_update(const Geometry& g, const CgState& s, int u, int steps, int fixed,
                            int split, hipStream_t st);
// Writes the probe key of an E-step to the device word keyp (one thread).
hipError_t launch_set_key(uint64_t* keyp, uint64_t key, hipStream_t st);
template <typename VT>
hipError_t launch_estep_finalize(const Geometry& g, const CgState& s, int K, const uint64_t* keyp,
                                 const int8_t* probes, int crn, float* mu, float* sdiag,
                                 hipStream_t st);
template <typename VT>
hipError_t launch_solve_output(const Geometry& g, const CgState& s, void* X, double* gam_out,
                               double* xi_out, int steps, int* iters_out, uint8_t* status_out,
                               hipStream_t st);
// colc: [T][Rp] cluster of every column slot (-1 for padding).  host_map: [T][R] or null
// (then slot j of every task belongs to cluster j / (K+1)).
hipError_t launch_fill_colc(int* colc, int T, int R, int Rp, int K, const int32_t* host_map,
                            hipStream_t st);
template <typename VT>
hipError_t launch_pack2(const Geometry& g, const void* X, const void* Lam, void* Dv,
                        hipStream_t st);
template <typename VT>
hipError_t launch_grads(const Geometry& g, int R, const VT* XL, const VT* W, const float* y,
                        const int* colc, double beta, double y_coef, float* dalpha,
                        float* dphi, int64_t rows, hipStream_t st);
hipError_t launch_zero_i32(int* p, long n, hipStream_t st);
// Per-right-hand-side statistics of an E-step: iters and status ([T][R]; probe columns whose
// tridiagonal was not certified positive definite, ok[p] = 0, get CMTCS_CG_NONPOS_RITZ) and the
// number of probes K_eff of each (t, c) that entered nu ([T][C]).  Each output may be null.
hipError_t launch_stats_estep(const Geometry& g, const CgState& s, int K, const uint8_t* ok,
                              const int* keff, int32_t* iters_out, uint8_t* status_out,
                              int32_t* keff_out, hipStream_t st);

// Launchers (k_slq.hip).
// steps: the largest number of CG steps any probe took (bounds the tridiagonal size).
// The tridiagonals of up to four probes share a block's LDS while they fit in lds_bytes (at
// most kSlqLdsBytes); longer runs keep them in rows_ws, a device workspace of
// slq_workspace_bytes(T*C*K, steps, lds_bytes) bytes (none when they fit).  Both forms give
// identical results.
constexpr long kSlqLdsBytes = 64 * 1024;
size_t slq_workspace_bytes(long P, int steps, long lds_bytes);
hipError_t launch_slq(const Geometry& g, const CgState& s, int K, int steps, double pnorm2,
                      void* rows_ws, double* tau, uint8_t* ok, double* rmin, double* rmax,
                      long lds_bytes, hipStream_t st);

// Launchers (k_mixed.hip).  g16.w_off holds the offsets of the 16-bit W (rows padded to 32).
// which: 1 = the Phi V16 product only, 2 = the Phi^T W16 product only.
template <typename T16>
hipError_t launch_mixed_products(const Geometry& g16, const void* phi16, const void* phiT16,
                                 const int4* fwd, int nfwd, const int4* adj, int nadj,
                                 const void* V16, void* W16, const float* V, float* AV,
                                 const float* alpha, const int* colc, double beta,
                                 const int* act, int which, hipStream_t st);
template <typename T16>
hipError_t launch_transpose16(const Geometry& g16, const void* phi16, void* phiT16, int max_np,
                              hipStream_t st);
// y[r][c] = round16(x[r][c]) for rows x cols, row pitches ldx and ldy (elements).
template <typename T16>
hipError_t launch_round16(const float* x, int64_t ldx, void* y, int64_t ldy, int64_t rows,
                          int cols, hipStream_t st);
// Second half of a residual-replacement step u: r = src - A x (A x in AX), then r.r, xi,
// d = r + xi d and the stop decision of the step, as in the unsplit update.
hipError_t launch_replace(const Geometry& g, const CgState& s, const float* AX,
                          const RhsSource& src, int u, int steps, int fixed, hipStream_t st);
constexpr int kRows16 = 64;   // output rows per wave tile of the 16-bit products
// Row pitch (elements) of the 16-bit arrays of the mixed path for rows of n elements: 128 bytes
// past a multiple of 256.  Many waves read their rows in step, so rows that all start on the
// same power-of-two boundary put the reads of a step on the same few memory channels (measured:
// 4.3 TB/s for 64-row tiles at an 8 KB pitch, 6.1 TB/s at 8 KB + 128 B, like a linear stream).
__host__ __device__ constexpr int64_t ld16(int64_t n) { return (n + 127) / 128 * 128 + 64; }

// Launchers (k_fourier.hip): partial-Fourier problems (D a power of two, 64..4096, FP64).
// mode 0: the whole CG solve of every column (two columns per workgroup), writing X, the
// gamma/xi histories, iters and state of s; mode 1: X = A B for the columns of src.B (kind 1).
hipError_t launch_fourier_cg(const Geometry& g, const CgState& s, const int* hcount, int mode,
                             const RhsSource& src, double tol, int steps, int fixed,
                             hipStream_t st);
// b = beta Re(F^H Omega^T y) per task and hcount[t][k] = m_k + m_{-k}; frequencies outside
// [0, D) are counted in *bad.
hipError_t launch_fourier_setup(const Geometry& g, const int* freq, const float* yc, double beta,
                                double* b, int* hcount, int* bad, hipStream_t st);

// Launchers (k_em.hip).
template <typename VT>
hipError_t launch_rhs(const Geometry& g, const float* phi, const float* y, double beta, VT* b,
                      hipStream_t st);
hipError_t launch_sum_log_alpha(int C, int D, const float* alpha, double* slog, hipStream_t st);
// Jacobi preconditioner of an E-step or solve: mdiag[t][c][d] = mbase[t][d] + alpha[c][d]
// (mbase = beta diag(Phi_t^T Phi_t), computed once per handle by launch_colnorm) and
// slogm[t][c] = sum_d log mdiag[t][c][d].
hipError_t launch_colnorm(const Geometry& g, const float* phi, double beta, double* mbase,
                          hipStream_t st);
hipError_t launch_jacobi(const Geometry& g, const double* mbase, const float* alpha,
                         double* mdiag, double* slogm, hipStream_t st);

template <typename VT>
hipError_t launch_resp(const Geometry& g, const CgState& s, int K, const VT* b,
                       const double* tau, const uint8_t* ok, const double* slog,
                       const double* log_pi, double* logdet, double* ell, double* q,
                       int* keff, const double* slogm, hipStream_t st);
hipError_t launch_mstep(int T, int C, int D, const float* mu, const float* sdiag,
                        const double* q, double alpha_max, float* alpha, hipStream_t st);
hipError_t launch_update_pi(int T, int C, const double* q, double* log_pi, hipStream_t st);
// const_t of the marginal likelihood per task (per_row real values per stored measurement row)
hipError_t launch_log_norm_const(int T, const float* y, const int64_t* row_off, int per_row,
                                 double beta, double* lconst, hipStream_t st);
// L_t and their mean from ell [T][C] and log_pi [C]; Lt and L may be null
hipError_t launch_log_likelihood(int T, int C, const double* ell, const double* log_pi,
                                 const double* lconst, double* Lt, double* L, hipStream_t st);

}  // namespace cmtcs
