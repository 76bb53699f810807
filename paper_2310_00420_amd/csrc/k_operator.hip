// Matrix-free operator of CoFEM: for every task t, A_tc V = beta Phi_t^T (Phi_t V) + alpha_c (.) V
// applied to all right-hand sides of the task at once (Sec. 3.3: only products with Phi and
// Phi^T are needed, A is never formed).  Two matrix-core products per CG step:
//
//   fwd:  W_t  = Phi_t V_t          W_t [Rp][np_t], contraction over d (both operands
//                                    d-contiguous: Phi_t rows and V_t columns)
//   adj:  AV_t = beta Phi_t^T W_t + alpha_{c(j)} (.) V_t     contraction over n
//         (or the bare Phi_t^T W_t when no alpha is given: the CG update then adds beta and
//         the diagonal term while it reads V_t anyway)
//
// Each wave owns one output tile (16*RF rows x up to 144 columns) and keeps the whole
// contraction in accumulator registers.  Loads are 16-byte or wider: lane l of the wave reads
// consecutive elements of one row, and the four k-steps of a 16x16x4 tile take the four
// consecutive elements in turn (a permutation of the contraction index that both operands
// share, so the sum is unchanged).  Phi is streamed once per tile from HBM; the shared
// right-hand-side block (V_t or W_t) is re-read by all tiles of a task and stays in L2, which is
// why the block index is remapped so that the tiles of one task run on the same XCD.
#include <type_traits>
#include <utility>

#include "internal.h"

namespace cmtcs {

// Workgroups are dispatched round-robin over the 8 XCDs; map the hardware block index to a
// logical one so that each XCD receives a contiguous range of logical blocks.
__device__ inline int xcd_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, rem) + i;
}

// Compaction of a task's right-hand sides in the CG loop.  Column positions 0 .. nact-1 of task
// t list its active slots (state kActive) in increasing order; the remaining positions hold its
// stopped and padding slots, from the last position down.  A tile of column group g multiplies
// the fragments that hold positions 16 kColGroup g .. up to the last active one, so fragments
// whose columns have all stopped (and, once a task has fewer active columns, the padding
// fragment) cost nothing.  The forward product reads V at the slots and writes W by position;
// the adjoint reads W by position and writes at the slots.  Every output column is the same
// sequence of operations whichever fragment holds it, so the results do not depend on the
// compaction.  One wave scans the task's states (64 a round, by ballot) and stores
// map[i] = slot of position p0 + i for 0 <= i < 16 kColGroup (if `store`); it returns nact.
__device__ inline int col_map(const uint8_t* __restrict__ state, int t, int Rp, int p0,
                              int* __restrict__ map, bool store = true) {
  const int lane = threadIdx.x & 63;
  const uint8_t* st = state + (int64_t)t * Rp;
  const uint64_t lt = lane == 0 ? 0ull : ~0ull >> (64 - lane);
  int nact = 0, nstop = 0;
  for (int base = 0; base < Rp; base += 64) {
    const int j = base + lane;
    const bool valid = j < Rp;
    const bool a = valid && st[j] == kActive;
    const uint64_t ma = __ballot(a), ms = __ballot(valid && !a);
    const int p = a ? nact + __popcll(ma & lt) : Rp - 1 - (nstop + __popcll(ms & lt));
    const int i = p - p0;
    if (store && valid && i >= 0 && i < 16 * kColGroup) map[i] = j;
    nact += __popcll(ma);
    nstop += __popcll(ms);
  }
  return uniform(nact);
}

// Column fragments a tile of the group starting at fragment cf0 multiplies: all of the group,
// or with a column map those up to the last active position.
__device__ inline int active_frags(int ncf, int cf0, int nact) {
  return min(ncf, (nact - 16 * cf0 + 15) >> 4);
}

// Whether the last fragment a tile multiplies holds at most four active positions: the
// LDS-staged FP64 kernels then multiply only its first four columns, with 4x4x4 products (a
// quarter of the work; the other twelve are stopped or padding columns, whose outputs nothing
// reads).
__device__ inline bool narrow_last(int ncf, int cf0, int nact) {
  return nact - 16 * (cf0 + ncf - 1) <= 4;
}
template <typename VT, int RF>
constexpr bool kNarrowOk = sizeof(VT) == 8 && RF == 1;

// Makes one wave's LDS stores visible to its own later LDS loads.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Output rows per wave tile (16 * RF) that the instantiations below support; the autotuner of
// the host layer picks one per product.  FP64 tiles keep RF * 9 accumulators of 8 registers.
// Waves (tiles) per workgroup.  Four measured faster than one on the FP64 tiles, although a
// SIMD then starts its next tile only when all four waves of its group have ended.
constexpr int kOpWaves = 4;

// Depth of the register ring that prefetches the Phi operand (depth - 1 chunks ahead), per
// element type of the right-hand sides: measured best at 6 for FP64 (8 spills) and 4 for FP32.
template <typename VT> constexpr int ring_depth() { return sizeof(VT) == 8 ? 6 : 4; }

// The LDS-staged kernels (two waves per SIMD) are offered as 16-row FP64 tiles for both
// products and as 32-row FP32 tiles for the adjoint product: at the precision and batching
// workloads the autotuner keeps them.  With 32 FP64 rows an LDS-staged kernel stays at one wave
// per SIMD and loses; for the FP32 forward product the register-pipelined 64-row tile is faster.
int op_row_candidates(bool f64, int kind, int* rows) {
  if (!f64) {   // the first entry is the default
    rows[0] = 64; rows[1] = 32;
    if (kind == 0) {
      // 16-row forward tiles for short tasks: N_t = 256 gives 16 tiles per task instead of 8
      rows[2] = 16;
      return 3;
    }
    rows[2] = -32;
    return 3;
  }
  rows[0] = 32; rows[1] = 16; rows[2] = -16;
  return 3;
}

// KSPL = 1: each wave of a block owns a tile.  KSPL = kOpWaves: the block owns one tile and its
// waves split the contraction over d, wave w taking chunks [w nch / KSPL, (w + 1) nch / KSPL);
// waves 1.. leave their sums in LDS and wave 0 adds them in wave order before the epilogue.
template <typename VT, int RF, int KSPL = 1>
__global__ __launch_bounds__(64 * kOpWaves) void k_phi_v(const float* __restrict__ phi,
                                               const int64_t* __restrict__ row_off,
                                               const int64_t* __restrict__ w_off,
                                               const int4* __restrict__ tiles, int ntiles,
                                               const VT* __restrict__ V, VT* __restrict__ W,
                                               const int* __restrict__ act,
                                               const uint8_t* __restrict__ state, int D, int Rp) {
  typedef typename Mfma<VT>::acc_t acc_t;
  typedef typename VecOf<VT, 4>::type vt4;
  constexpr int kRingA = ring_depth<VT>();
  static_assert(KSPL == 1 || KSPL == kOpWaves, "one tile per wave or per block");
  __shared__ int cmap[kOpWaves][16 * kColGroup];
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, g4 = lane >> 4;
  // tile fields are wave-uniform: keep them in scalar registers so that every branch on them
  // is a scalar branch, not an exec-mask branch around matrix-core instructions.  With the
  // split every return below is uniform over the block (its waves share the tile), so that
  // all of them reach the barriers of the reduction or none does.
  const int tile = KSPL > 1
      ? uniform(xcd_block(blockIdx.x, gridDim.x))
      : uniform(xcd_block(blockIdx.x, gridDim.x) * kOpWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int4 tl = tiles[tile];
  const int t = uniform(tl.x), n0 = uniform(tl.y), cf0 = uniform(tl.z) * kColGroup;
  if (act != nullptr && act[t] == 0) return;
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (int)((w_off[t + 1] - w_off[t]) / Rp);
  int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  int* map = cmap[threadIdx.x >> 6];
  if (state != nullptr) {
    ncf = active_frags(ncf, cf0, col_map(state, t, Rp, 16 * cf0, map));
    if (ncf <= 0) return;
    wave_lds_sync();
  }

  // Phi rows of the task and V_t through buffer descriptors (per-lane 32-bit byte offsets, the
  // chunk's start as a scalar offset).  Matrix row i16 of fragment rf is Phi row
  // n0 + rf*16 + a_row(i16), so that the accumulator of lane (g4, r) holds the consecutive rows
  // n0 + rf*16 + 4 g4 + r.  Rows past N_t lie past the descriptor's end and read as zeros; the
  // epilogue writes their outputs as zeros anyway.
  const rsrc_t rphi = make_rsrc(phi + r0 * (int64_t)D, (uint32_t)((int64_t)nt * D * 4));
  uint32_t aoff[RF];
#pragma unroll
  for (int rf = 0; rf < RF; ++rf)
    aoff[rf] = (uint32_t)(((n0 + rf * 16 + Mfma<VT>::a_row(i16)) * D + 4 * g4) * 4);
  const rsrc_t rv = make_rsrc(V + (int64_t)t * Rp * D, (uint32_t)((int64_t)Rp * D * sizeof(VT)));
  // V column of lane i16 in fragment f: its slot (position cf0*16 + f*16 + i16)
  uint32_t boff[kColGroup];
#pragma unroll
  for (int f = 0; f < kColGroup; ++f) {
    const int pos = min(f, ncf - 1) * 16 + i16;
    const int slot = state != nullptr ? map[pos] : cf0 * 16 + pos;
    boff[f] = (uint32_t)((slot * D + 4 * g4) * sizeof(VT));
  }

  acc_t acc[RF][kColGroup];
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int rf = 0; rf < RF; ++rf)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf) acc[rf][cf] = acc_t{0, 0, 0, 0};
  };

  // Software pipeline over chunks of 16 along d.  The Phi operand streams from HBM (it misses
  // L2 every time), so it is prefetched kRingA - 1 chunks ahead in a ring of register buffers;
  // the right-hand-side block comes from L2 and is double-buffered one chunk ahead.  Every load
  // is unconditional and no loaded value is touched before its MFMA; a load past the last chunk
  // re-reads the last chunk (in bounds, unused) and a missing column fragment re-reads the last
  // present one.  In each slot the right-hand-side loads are issued before the Phi loads: the
  // memory counter completes in issue order, so waiting for a chunk's right-hand side then
  // does not also wait for the Phi loads of later chunks.
  // this wave's chunks: cb .. cb + nch - 1 (all D / 16 of them without the split)
  const int wv = KSPL > 1 ? uniform(threadIdx.x >> 6) : 0;
  const int cb = KSPL > 1 ? uniform(wv * (D / 16) / KSPL) : 0;
  const int nch = KSPL > 1 ? uniform((wv + 1) * (D / 16) / KSPL) - cb : D / 16;
  // a chunk index past the wave's last (or any, for a wave without chunks) re-reads the last
  // one, or the range's first: in bounds, unused
  const int clast = KSPL > 1 ? cb + max(nch - 1, 0) : nch - 1;
  f4 a[kRingA][RF];
  vt4 b[2][kColGroup];
  auto load_a = [&](f4 (&x)[RF], int c) __attribute__((always_inline)) {
    const uint32_t soff = (uint32_t)uniform(min(cb + c, clast) * 64);
#pragma unroll
    for (int rf = 0; rf < RF; ++rf) x[rf] = buf_load<f4>(rphi, aoff[rf], soff);
  };
  // nf: the fragment count when it is a compile-time 9 or 8 (the common counts with
  // compaction), or 0 for any other count, then guarded at run time
  auto load_b = [&](vt4 (&x)[kColGroup], int c, auto nf) __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
    const uint32_t soff = (uint32_t)uniform(min(cb + c, clast) * 16 * (int)sizeof(VT));
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf)
      if (NF == 0 || cf < NF) x[cf] = buf_load<vt4>(rv, boff[cf], soff);
  };
  // first: the chunk that starts the accumulation (its first k-step takes a zero accumulator)
  auto mma = [&](const f4 (&x)[RF], const vt4 (&y)[kColGroup], auto nf, auto first)
      __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf)
        if (NF == 0 ? cf < ncf : cf < NF)
#pragma unroll
          for (int rf = 0; rf < RF; ++rf) {
            const acc_t cin = (decltype(first)::value && s == 0) ? acc_t{0, 0, 0, 0} : acc[rf][cf];
            acc[rf][cf] = Mfma<VT>::mma((VT)x[rf][s], y[cf][s], cin);
          }
  };
  auto slot = [&](int c, auto ic, auto nf, auto first) __attribute__((always_inline)) {
    constexpr int i = decltype(ic)::value;
    load_b(b[(i + 1) & 1], c + i + 1, nf);
    load_a(a[(i + kRingA - 1) % kRingA], c + i + kRingA - 1);
    // the scheduling barriers keep the compiler from moving loads across the MFMAs they
    // should overlap, or conversions up to their loads
    __builtin_amdgcn_sched_barrier(0);
    mma(a[i], b[i & 1], nf, first);
    __builtin_amdgcn_sched_barrier(0);
  };
  auto ring = [&](int c, auto nf, auto first) __attribute__((always_inline)) {
    static_for<kRingA>([&](auto ic) __attribute__((always_inline)) {
      slot(c, ic, nf,
           std::integral_constant<bool, decltype(first)::value && decltype(ic)::value == 0>{});
    });
  };
  auto run = [&](auto nf) __attribute__((always_inline)) {
    load_b(b[0], 0, nf);
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) load_a(a[i], i);
    int c = 0;
    if (nch >= kRingA) {
      // rounds of kRingA chunks; the first is peeled so that the accumulators start in the
      // matrix-core result registers (a zero input to the first k-step) instead of as zeros
      // carried into the loop, which made the compiler copy them across every iteration
      ring(0, nf, std::true_type{});
      for (c = kRingA; c + kRingA <= nch; c += kRingA) ring(c, nf, std::false_type{});
    } else {
      zero_acc();
    }
    // fewer than kRingA chunks left: chunk c+i is in a[i], chunk c's right-hand side in b[0]
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) {
      if (c + i >= nch) break;
      if (i > 0) load_b(b[i & 1], c + i, nf);
      mma(a[i], b[i & 1], nf, std::false_type{});
    }
  };
  if (ncf == kColGroup) run(std::integral_constant<int, kColGroup>{});   // no guards
  else if (ncf == kColGroup - 1) run(std::integral_constant<int, kColGroup - 1>{});
  else run(std::integral_constant<int, 0>{});

  if constexpr (KSPL > 1) {
    // wave 0 adds the sums of waves 1, 2, .. (in that order), one row fragment at a time;
    // every wave passes the same 2 RF barriers
    __shared__ acc_t red[(KSPL - 1) * kColGroup * 64];
#pragma unroll
    for (int rf = 0; rf < RF; ++rf) {
      if (wv > 0) {
#pragma unroll
        for (int cf = 0; cf < kColGroup; ++cf)
          if (cf < ncf) red[((wv - 1) * kColGroup + cf) * 64 + lane] = acc[rf][cf];
      }
      __syncthreads();
      if (wv == 0) {
#pragma unroll
        for (int w = 1; w < KSPL; ++w)
#pragma unroll
          for (int cf = 0; cf < kColGroup; ++cf)
            if (cf < ncf) acc[rf][cf] = acc[rf][cf] + red[((w - 1) * kColGroup + cf) * 64 + lane];
      }
      __syncthreads();
    }
    if (wv > 0) return;
  }

  VT* Wt = W + w_off[t];
#pragma unroll
  for (int rf = 0; rf < RF; ++rf) {
    const int rb = n0 + rf * 16;
    if (rb >= np) continue;
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (cf >= ncf) continue;
      const int j = (cf0 + cf) * 16 + i16;
      // rows N_t..np-1 of W are zero: the adjoint product contracts over them
      vt4 o;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = rb + 4 * g4 + r < nt ? (VT)acc[rf][cf][r] : (VT)0;
      *(vt4*)(Wt + (int64_t)j * np + rb + 4 * g4) = o;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// LDS-staged forward product.  A block of four waves owns four consecutive 16*RF-row tiles of
// one task and one column group, so all four multiply the same right-hand-side chunk: the block
// loads it once per chunk into an LDS double buffer (through a few staging registers per
// thread) instead of each wave loading it into its own registers.  The Phi ring and the
// accumulators are per wave as in k_phi_v.
//
// Layout of a staged chunk in LDS (16 elements along the contraction x up to 144 columns).  The
// matrix-core operand of lane (i16, g4) is column i16 of a fragment at elements 4 g4 .. 4 g4 + 3,
// read 16 bytes at a time.  Measured on gfx950 (bank-conflict counters on probe kernels): a
// 16-byte LDS read is conflict-free when each 16-lane quarter of the wave reads one aligned
// 256-byte block, and a 16-byte write when the 8 lanes of each eighth fall in distinct banks of
// a 128-byte row.  FP64 therefore stores a fragment's chunk piece-major: 16-byte piece q (two
// elements) of column c at 16 q + (c ^ q) pieces into the fragment's 2 KB, so that a quarter
// wave reads piece q of all 16 columns (one 256-byte row, permuted) and the staging stores,
// where 8 lanes write pieces 0..7 of one column, land in 8 different banks.  (Columns as padded
// rows of 18 elements cost 4 conflict cycles on every operand read.)  FP32, whose operand reads
// are 8 bytes, keeps the padded rows.
template <typename VT>
struct LdsChunk {
  static constexpr int kPer16 = 16 / (int)sizeof(VT);            // elements per 16-byte piece
  static constexpr int kPieces = 16 / kPer16;                    // pieces per 16-element column
  static constexpr int kLd = 16 + kPer16;                        // padded LDS row (elements)
  static constexpr int kMaxPieces = 16 * kColGroup * kPieces;
  static constexpr int kPerThread = (kMaxPieces + 64 * kOpWaves - 1) / (64 * kOpWaves);
  static constexpr bool kSwizzled = sizeof(VT) == 8;
  static constexpr int kBufElems = kSwizzled ? kColGroup * 16 * 16 : 16 * kColGroup * kLd;
  typedef typename VecOf<VT, kPer16>::type piece_t;
  // element offset, within one buffer, of element e (e even for FP64) of column col
  __device__ static inline int off(int col, int e) {
    if constexpr (kSwizzled) {
      const int q = e >> 1;
      return ((((col >> 4) << 7) + (q << 4) + ((col & 15) ^ q)) << 1) + (e & 1);
    } else {
      return col * kLd + e;
    }
  }
};

// The 16-row FP64 LDS-staged tile fits two waves per SIMD without spilling once the
// right-hand side no longer sits in registers (larger tiles do not).
template <typename VT, int RF>
constexpr int lds_waves_per_simd() { return (sizeof(VT) == 8 ? RF == 1 : RF == 2) ? 2 : 1; }

template <typename VT, int RF>
__global__ __launch_bounds__(64 * kOpWaves, (lds_waves_per_simd<VT, RF>())) void k_phi_v_lds(const float* __restrict__ phi,
                                                   const int64_t* __restrict__ row_off,
                                                   const int64_t* __restrict__ w_off,
                                                   const int4* __restrict__ tiles, int ntiles,
                                                   const VT* __restrict__ V, VT* __restrict__ W,
                                                   const int* __restrict__ act,
                                                   const uint8_t* __restrict__ state, int D,
                                                   int Rp) {
  typedef typename Mfma<VT>::acc_t acc_t;
  typedef typename VecOf<VT, 4>::type vt4;
  typedef LdsChunk<VT> L;
  typedef typename L::piece_t piece_t;
  // four chunks in the Phi ring (three ahead): with the per-count instantiations six spilled
  constexpr int kRingA = 4;
  __shared__ VT lds[2 * L::kBufElems];
  __shared__ int cmap[16 * kColGroup];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int blk = uniform(xcd_block(blockIdx.x, gridDim.x));
  if (blk >= ntiles) return;
  const int4 tl = tiles[blk];
  const int t = uniform(tl.x), cf0 = uniform(tl.z) * kColGroup;
  const int n0 = uniform(tl.y) + uniform(wave) * 16 * RF;
  if (act != nullptr && act[t] == 0) return;   // uniform over the block
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (int)((w_off[t + 1] - w_off[t]) / Rp);
  int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  bool narrow = false;
  if (state != nullptr) {
    // every wave scans (the same count); wave 0 stores the map
    const int nact = col_map(state, t, Rp, 16 * cf0, cmap, wave == 0);
    ncf = active_frags(ncf, cf0, nact);
    if (ncf <= 0) return;   // uniform over the block
    if constexpr (kNarrowOk<VT, RF>) narrow = narrow_last(ncf, cf0, nact);
    __syncthreads();
  }

  // as in k_phi_v: Phi through a buffer descriptor; rows past N_t (also whole tiles of the
  // block past np) read as zeros and their outputs are zeroed or not stored
  const rsrc_t rphi = make_rsrc(phi + r0 * (int64_t)D, (uint32_t)((int64_t)nt * D * 4));
  uint32_t aoff[RF];
#pragma unroll
  for (int rf = 0; rf < RF; ++rf)
    aoff[rf] = (uint32_t)(((n0 + rf * 16 + Mfma<VT>::a_row(i16)) * D + 4 * g4) * 4);
  // staging: piece p of the chunk is column p / kPieces, 16-byte piece p % kPieces; pieces past
  // the group's columns are clamped onto the last one (a duplicate load and an identical store)
  const int npieces = (16 * ncf - (narrow ? 12 : 0)) * L::kPieces;
  const rsrc_t rv = make_rsrc(V + (int64_t)t * Rp * D, (uint32_t)((int64_t)Rp * D * sizeof(VT)));
  uint32_t soff_v[L::kPerThread];
  VT* sdst[2][L::kPerThread];
#pragma unroll
  for (int i = 0; i < L::kPerThread; ++i) {
    const int p = min((int)threadIdx.x + i * 64 * kOpWaves, npieces - 1);
    const int col = p / L::kPieces, q = p % L::kPieces;
    const int slot = state != nullptr ? cmap[col] : cf0 * 16 + col;
    soff_v[i] = (uint32_t)((slot * D + q * L::kPer16) * sizeof(VT));
    sdst[0][i] = &lds[L::off(col, q * L::kPer16)];
    sdst[1][i] = &lds[L::kBufElems + L::off(col, q * L::kPer16)];
  }

  acc_t acc[RF][kColGroup];
  VT acc4 = 0;   // the narrow last fragment
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int rf = 0; rf < RF; ++rf)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf) acc[rf][cf] = acc_t{0, 0, 0, 0};
    acc4 = 0;
  };

  const int nch = D / 16;
  f4 a[kRingA][RF];
  piece_t stg[L::kPerThread];
  auto load_a = [&](f4 (&x)[RF], int c) __attribute__((always_inline)) {
    const uint32_t soff = (uint32_t)uniform(min(c, nch - 1) * 64);
#pragma unroll
    for (int rf = 0; rf < RF; ++rf) x[rf] = buf_load<f4>(rphi, aoff[rf], soff);
  };
  auto stage_load = [&](int c) __attribute__((always_inline)) {
    const uint32_t soff = (uint32_t)uniform(min(c, nch - 1) * 16 * (int)sizeof(VT));
#pragma unroll
    for (int i = 0; i < L::kPerThread; ++i) stg[i] = buf_load<piece_t>(rv, soff_v[i], soff);
  };
  auto stage_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < L::kPerThread; ++i) *(piece_t*)sdst[buf][i] = stg[i];
  };
  // the right-hand-side fragments are read in two halves (k-steps 0-1, then 2-3), which halves
  // the registers they hold; the products run in the same order as in k_phi_v
  typedef typename VecOf<VT, 2>::type vt2;
  // nw: the last fragment is narrow (4x4x4 products on its first four columns; FP64, RF = 1)
  auto step = [&](const f4 (&x)[RF], int buf, auto nf, auto nw, auto first)
      __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
    constexpr bool kNw = decltype(nw)::value;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      vt2 b[kColGroup];
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf)
        if (cf < NF)
          b[cf] = *(const vt2*)&lds[buf * L::kBufElems +
                                    L::off(cf * 16 + ((kNw && cf == NF - 1) ? (i16 & 3) : i16),
                                           4 * g4 + 2 * h)];
#pragma unroll
      for (int ss = 0; ss < 2; ++ss) {
        const int s = 2 * h + ss;
#pragma unroll
        for (int cf = 0; cf < kColGroup; ++cf)
          if (cf < NF) {
            if constexpr (kNw) {
              if (cf == NF - 1) {
                acc4 = mma4<VT>((VT)x[0][s], b[cf][ss],
                                (decltype(first)::value && s == 0) ? (VT)0 : acc4);
                continue;
              }
            }
#pragma unroll
            for (int rf = 0; rf < RF; ++rf) {
              const acc_t cin = (decltype(first)::value && s == 0) ? acc_t{0, 0, 0, 0} : acc[rf][cf];
              acc[rf][cf] = Mfma<VT>::mma((VT)x[rf][s], b[cf][ss], cin);
            }
          }
      }
    }
  };
  // Per chunk c (buffer c & 1): multiply; store the staged chunk c+1 into the other buffer
  // (whose chunk c-1 every wave finished before the last barrier); stage chunk c+2; then the
  // Phi load of chunk c + kRingA - 1, issued after the staging loads so that the next wait for
  // staged data does not also wait for it; barrier.
  auto chunk = [&](int c, auto ic, auto nf, auto nw, auto first) __attribute__((always_inline)) {
    constexpr int i = decltype(ic)::value;
    step(a[i], i & 1, nf, nw, first);
    stage_store((i + 1) & 1);
    stage_load(c + i + 2);
    load_a(a[(i + kRingA - 1) % kRingA], c + i + kRingA - 1);
    __syncthreads();
  };
  auto ring = [&](int c, auto nf, auto nw, auto first) __attribute__((always_inline)) {
    static_for<kRingA>([&](auto ic) __attribute__((always_inline)) {
      chunk(c, ic, nf, nw,
            std::integral_constant<bool, decltype(first)::value && decltype(ic)::value == 0>{});
    });
  };
  auto run = [&](auto nf, auto nw) __attribute__((always_inline)) {
    stage_load(0);
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) load_a(a[i], i);
    stage_store(0);
    stage_load(1);
    __syncthreads();
    int c = 0;
    if (nch >= kRingA) {   // kRingA is even: chunk c + i is in buffer i & 1
      // first round peeled so that the accumulators start in the matrix-core result registers
      ring(0, nf, nw, std::true_type{});
      for (c = kRingA; c + kRingA <= nch; c += kRingA) ring(c, nf, nw, std::false_type{});
    } else {
      zero_acc();
    }
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) {
      if (c + i >= nch) break;
      step(a[i], i & 1, nf, nw, std::false_type{});
      stage_store((i + 1) & 1);
      stage_load(c + i + 2);
      __syncthreads();
    }
  };
  // one instantiation per fragment count (and narrow last fragment), chosen once per tile:
  // guards on a run-time count inside the pipeline cost more than the skipped products save
  static_for<kColGroup>([&](auto i) __attribute__((always_inline)) {
    constexpr int NF = decltype(i)::value + 1;
    if (ncf != NF) return;
    if constexpr (kNarrowOk<VT, RF>) {
      if (narrow) {
        run(std::integral_constant<int, NF>{}, std::true_type{});
        return;
      }
    }
    run(std::integral_constant<int, NF>{}, std::false_type{});
  });

  VT* Wt = W + w_off[t];
#pragma unroll
  for (int rf = 0; rf < RF; ++rf) {
    const int rb = n0 + rf * 16;
    if (rb >= np) continue;
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (cf >= ncf) continue;
      if constexpr (kNarrowOk<VT, RF>) {
        if (narrow && cf == ncf - 1) {
          // one value per lane: row narrow_row, column i16 & 3 (Phi row order as in a_row)
          const int row = rb + Mfma<VT>::a_row(narrow_row(i16, g4));
          Wt[(int64_t)((cf0 + cf) * 16 + (i16 & 3)) * np + row] = row < nt ? acc4 : (VT)0;
          continue;
        }
      }
      const int j = (cf0 + cf) * 16 + i16;
      vt4 o;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = rb + 4 * g4 + r < nt ? (VT)acc[rf][cf][r] : (VT)0;
      *(vt4*)(Wt + (int64_t)j * np + rb + 4 * g4) = o;
    }
  }
}

// Epilogue of the adjoint product for one wave's tile (rows d0 .. d0 + 16 RF - 1 of task t,
// column fragments cf0 .. cf0 + ncf - 1): with no alpha the bare Phi^T W, else
// beta Phi^T W + alpha_c (.) V with one explicit fused multiply-add per element.
template <typename VT, int RF>
__device__ inline void phit_w_store(const typename Mfma<VT>::acc_t (&acc)[RF][kColGroup], int t,
                                    int d0, int cf0, int ncf, int i16, int g4, int D, int Rp,
                                    VT* __restrict__ AV, const VT* __restrict__ V,
                                    const float* __restrict__ alpha,
                                    const int* __restrict__ colc, double beta,
                                    const int* __restrict__ map) {
  typedef typename VecOf<VT, RF>::type vrf;
  // output column of lane i16 in fragment cf: position (cf0 + cf) * 16 + i16, at its slot
  auto slot_of = [&](int cf) __attribute__((always_inline)) {
    return map != nullptr ? map[cf * 16 + i16] : (cf0 + cf) * 16 + i16;
  };
  if (alpha == nullptr) {
    // bare product Phi^T W (the CG update adds beta and the diagonal term): stores only, so
    // the epilogue issues no load and never waits on memory
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (cf >= ncf) continue;
      const int64_t col = ((int64_t)t * Rp + slot_of(cf)) * D;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = d0 + RF * Mfma<VT>::out_row(g4, r);
        if (d >= D) continue;
        if constexpr (RF == 1) {
          AV[col + d] = acc[0][cf][r];
        } else {
          vrf o;
#pragma unroll
          for (int f = 0; f < RF; ++f) o[f] = acc[f][cf][r];
          *(vrf*)(AV + col + d) = o;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int cf = 0; cf < kColGroup; ++cf) {
    if (cf >= ncf) continue;
    const int j = slot_of(cf);
    const int c = colc[(int64_t)t * Rp + j];
    const int64_t col = ((int64_t)t * Rp + j) * D;
    const float* al = alpha + (int64_t)(c >= 0 ? c : 0) * D;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = d0 + RF * Mfma<VT>::out_row(g4, r);
      if (d >= D) continue;
      // one explicit fused multiply-add per element, so that every tile shape rounds the
      // epilogue identically (results do not depend on the autotuner's choice)
      if constexpr (RF == 1) {
        const VT a = c >= 0 ? (VT)al[d] : (VT)0;
        const VT av = a * V[col + d];
        AV[col + d] = __builtin_fma((VT)beta, acc[0][cf][r], av);
      } else {
        const vrf v = *(const vrf*)(V + col + d);
        vrf o;
#pragma unroll
        for (int f = 0; f < RF; ++f) {
          const VT a = c >= 0 ? (VT)al[d + f] : (VT)0;
          const VT av = a * v[f];
          o[f] = __builtin_fma((VT)beta, acc[f][cf][r], av);
        }
        *(vrf*)(AV + col + d) = o;
      }
    }
  }
}

template <typename VT, int RF>
__global__ __launch_bounds__(64 * kOpWaves) void k_phit_w(const float* __restrict__ phi,
                                                const int64_t* __restrict__ row_off,
                                                const int64_t* __restrict__ w_off,
                                                const int4* __restrict__ tiles, int ntiles,
                                                const VT* __restrict__ W, const VT* __restrict__ V,
                                                VT* __restrict__ AV,
                                                const float* __restrict__ alpha,
                                                const int* __restrict__ colc, double beta,
                                                const int* __restrict__ act,
                                                const uint8_t* __restrict__ state, int D,
                                                int Rp) {
  typedef typename Mfma<VT>::acc_t acc_t;
  typedef typename VecOf<float, RF>::type frf;
  __shared__ int cmap[kOpWaves][16 * kColGroup];
  // k-steps of the 16x16x4 tiles per chunk (chunks of KC = 16 rows of n; 8-row chunks, with
  // 16-byte right-hand-side fragments, measured 2.5% slower in FP64)
  constexpr int KS = 4;
  constexpr int KC = 4 * KS;
  typedef typename VecOf<VT, KS>::type vtk;
  constexpr int kRingA = ring_depth<VT>();
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int tile = uniform(xcd_block(blockIdx.x, gridDim.x) * kOpWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int4 tl = tiles[tile];
  const int t = uniform(tl.x), d0 = uniform(tl.y), cf0 = uniform(tl.z) * kColGroup;
  if (act != nullptr && act[t] == 0) return;
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (int)((w_off[t + 1] - w_off[t]) / Rp);
  int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  int* map = nullptr;
  if (state != nullptr) {
    map = cmap[threadIdx.x >> 6];
    ncf = active_frags(ncf, cf0, col_map(state, t, Rp, 16 * cf0, map));
    if (ncf <= 0) return;
    wave_lds_sync();
  }
  const int dl = d0 + RF * i16;          // first of the RF output rows this lane loads
  // Phi rows of the task and W_t through buffer descriptors: per-lane 32-bit byte offsets,
  // the chunk's start in scalar registers.  Lanes past D read column 0 (outputs not stored).
  const float* phit = phi + r0 * (int64_t)D;
  uint32_t aoff[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) aoff[s] = (uint32_t)(((KS * g4 + s) * D + (dl < D ? dl : 0)) * 4);
  const rsrc_t rw = make_rsrc(W + w_off[t], (uint32_t)((int64_t)Rp * np * sizeof(VT)));
  const uint32_t boff0 = (uint32_t)(((cf0 * 16 + i16) * np + KS * g4) * sizeof(VT));
  const uint32_t bstep = (uint32_t)(16 * np * sizeof(VT));

  acc_t acc[RF][kColGroup];
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf) acc[f][cf] = acc_t{0, 0, 0, 0};
  };

  // Software pipeline as in k_phi_v, over chunks of KC rows of n (Phi kRingA - 1 chunks ahead,
  // W one; lane g4 takes rows KS g4 .. KS g4 + KS - 1 of a chunk in the KS k-steps).  The Phi
  // descriptor of a chunk starts at its first row and ends at row N_t, so rows past N_t read as
  // zeros (and would meet zero rows of W anyway).
  const int nch = np / KC;
  frf a[kRingA][KS];
  vtk b[2][kColGroup];
  auto load_a = [&](frf (&x)[KS], int c) __attribute__((always_inline)) {
    // a chunk starting past N_t gets length zero, so every lane reads zeros (a negative
    // length would wrap to an unchecked one)
    const int nb = uniform(min(c, nch - 1) * KC);
    const rsrc_t ra = make_rsrc(phit + (int64_t)nb * D,
                                (uint32_t)((int64_t)max(nt - nb, 0) * D * 4));
#pragma unroll
    for (int s = 0; s < KS; ++s) x[s] = buf_load<frf>(ra, aoff[s], 0);
  };
  // nf: the fragment count when it is a compile-time 9 or 8, else 0 (guarded at run time)
  auto load_b = [&](vtk (&x)[kColGroup], int c, auto nf) __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
    const uint32_t soff = (uint32_t)uniform(min(c, nch - 1) * KC * (int)sizeof(VT));
#pragma unroll
    for (int cf = 0; cf < kColGroup; ++cf) {
      if (NF != 0 && cf >= NF) continue;
      const int f = NF != 0 ? cf : min(cf, ncf - 1);
      x[cf] = buf_load<vtk>(rw, boff0 + (uint32_t)f * bstep, soff);
    }
  };
  // first: the chunk that starts the accumulation (its first k-step takes a zero accumulator)
  auto mma = [&](const frf (&x)[KS], const vtk (&y)[kColGroup], auto nf, auto first)
      __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf)
        if (NF == 0 ? cf < ncf : cf < NF)
#pragma unroll
          for (int f = 0; f < RF; ++f) {
            float av;
            if constexpr (RF == 1) av = x[s]; else av = x[s][f];
            const acc_t cin = (decltype(first)::value && s == 0) ? acc_t{0, 0, 0, 0} : acc[f][cf];
            acc[f][cf] = Mfma<VT>::mma((VT)av, y[cf][s], cin);
          }
  };
  // one slot of the pipeline: chunk c + i from ring entry i, loads for the chunks ahead
  auto slot = [&](int c, auto ic, auto nf, auto first) __attribute__((always_inline)) {
    constexpr int i = decltype(ic)::value;
    load_b(b[(i + 1) & 1], c + i + 1, nf);
    load_a(a[(i + kRingA - 1) % kRingA], c + i + kRingA - 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a[i], b[i & 1], nf, first);
    __builtin_amdgcn_sched_barrier(0);
  };
  auto ring = [&](int c, auto nf, auto first) __attribute__((always_inline)) {
    static_for<kRingA>([&](auto ic) __attribute__((always_inline)) {
      slot(c, ic, nf,
           std::integral_constant<bool, decltype(first)::value && decltype(ic)::value == 0>{});
    });
  };
  auto run = [&](auto nf) __attribute__((always_inline)) {
    if (nch < kRingA) {   // small task: a zero start and the tail alone
      zero_acc();
      if (nch == 0) return;   // empty task: the product is zero
    }
    load_b(b[0], 0, nf);
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) load_a(a[i], i);
    int c = 0;
    if (nch >= kRingA) {
      // the first round is peeled so that the accumulators start in the matrix-core result
      // registers (a zero input to the first k-step) rather than as zeros carried into the loop
      ring(0, nf, std::true_type{});
      for (c = kRingA; c + kRingA <= nch; c += kRingA) ring(c, nf, std::false_type{});
    }
    // fewer than kRingA chunks left: chunk c+i is in a[i], chunk c's right-hand side in b[0]
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) {
      if (c + i >= nch) break;
      if (i > 0) load_b(b[i & 1], c + i, nf);
      mma(a[i], b[i & 1], nf, std::false_type{});
    }
  };
  if (ncf == kColGroup) run(std::integral_constant<int, kColGroup>{});   // no guards
  else if (ncf == kColGroup - 1) run(std::integral_constant<int, kColGroup - 1>{});
  else run(std::integral_constant<int, 0>{});

  phit_w_store<VT, RF>(acc, t, d0, cf0, ncf, i16, g4, D, Rp, AV, V, alpha, colc, beta, map);
}

// LDS-staged adjoint product: as k_phi_v_lds for Phi^T W.  A block of four 16*RF-row waves
// owns 64*RF consecutive rows d of one task and column group; the chunk of W_t (16 rows of n x
// up to 144 columns) that all four multiply is staged once per block through an LDS double
// buffer, and the Phi operand (four rows of n per lane and chunk, RF consecutive d each) is
// prefetched per wave in a register ring, through a per-chunk descriptor as in k_phit_w.  The
// k-steps, accumulation order and epilogue are those of k_phit_w, so the results are the same.
// TR (RF = 1): the Phi operand comes from phiT, Phi_t transposed (D rows of np_t elements, rows
// N_t.. of Phi zero; task t at element D w_off[t] / Rp): the four rows of n a lane needs per
// chunk are then four consecutive elements, one 16-byte load instead of four 4-byte ones.  The
// same values reach the same matrix-core steps, so the results do not change.
template <typename VT, int RF, bool TR = false>
__global__ __launch_bounds__(64 * kOpWaves, (lds_waves_per_simd<VT, RF>())) void k_phit_w_lds(
    const float* __restrict__ phi, const int64_t* __restrict__ row_off,
    const int64_t* __restrict__ w_off, const int4* __restrict__ tiles, int ntiles,
    const VT* __restrict__ W, const VT* __restrict__ V, VT* __restrict__ AV,
    const float* __restrict__ alpha, const int* __restrict__ colc, double beta,
    const int* __restrict__ act, const uint8_t* __restrict__ state, int D, int Rp,
    const float* __restrict__ phiT) {
  static_assert(!TR || RF == 1, "the transposed operand serves one row per lane");
  typedef typename Mfma<VT>::acc_t acc_t;
  typedef typename VecOf<float, RF>::type frf;
  typedef LdsChunk<VT> L;
  typedef typename L::piece_t piece_t;
  constexpr int KS = 4;
  constexpr int KC = 4 * KS;   // rows of n per chunk (the 16-element columns of LdsChunk)
  // a shallower Phi ring than k_phit_w's: with the block sharing the W chunk, four entries keep
  // two waves per SIMD without spilling (six do not)
  constexpr int kRingA = 4;
  __shared__ VT lds[2 * L::kBufElems];
  __shared__ int cmap[16 * kColGroup];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int blk = uniform(xcd_block(blockIdx.x, gridDim.x));
  if (blk >= ntiles) return;
  const int4 tl = tiles[blk];
  const int t = uniform(tl.x), cf0 = uniform(tl.z) * kColGroup;
  const int d0 = uniform(tl.y) + uniform(wave) * 16 * RF;
  if (act != nullptr && act[t] == 0) return;   // uniform over the block
  const int64_t r0 = row_off[t];
  const int nt = (int)(row_off[t + 1] - r0);
  const int np = (int)((w_off[t + 1] - w_off[t]) / Rp);
  int ncf = uniform(min(kColGroup, Rp / 16 - cf0));
  const int* map = nullptr;
  bool narrow = false;
  if (state != nullptr) {
    // every wave scans (the same count); wave 0 stores the map
    const int nact = col_map(state, t, Rp, 16 * cf0, cmap, wave == 0);
    ncf = active_frags(ncf, cf0, nact);
    if (ncf <= 0) return;   // uniform over the block
    // the narrow fragment's outputs go through the bare-product store below
    if constexpr (kNarrowOk<VT, RF>) narrow = alpha == nullptr && narrow_last(ncf, cf0, nact);
    __syncthreads();
    map = cmap;
  }
  const int nch = np / KC;

  acc_t acc[RF][kColGroup];
  VT acc4 = 0;   // the narrow last fragment
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf) acc[f][cf] = acc_t{0, 0, 0, 0};
    acc4 = 0;
  };
  if (nch == 0) {   // empty task (uniform over the block): the product is zero
    zero_acc();
    phit_w_store<VT, RF>(acc, t, d0, cf0, ncf, i16, g4, D, Rp, AV, V, alpha, colc, beta, map);
    return;
  }
  // Phi as in k_phit_w: lanes past D read column 0 (outputs not stored); a chunk's descriptor
  // starts at its first row and ends at row N_t, so rows past N_t read as zeros
  const int dl = d0 + RF * i16;
  const float* phit = phi + r0 * (int64_t)D;
  // row KS*g4 + s of the chunk: one per-lane offset, the row step s*D as a scalar offset
  const uint32_t aoff0 = (uint32_t)((KS * g4 * D + (dl < D ? dl : 0)) * 4);
  // staging of W_t: piece p of the chunk is column p / kPieces, 16-byte piece p % kPieces;
  // pieces past the group's columns are clamped onto the last one
  const int npieces = (16 * ncf - (narrow ? 12 : 0)) * L::kPieces;
  const rsrc_t rw = make_rsrc(W + w_off[t], (uint32_t)((int64_t)Rp * np * sizeof(VT)));
  uint32_t soff_w[L::kPerThread];
  VT* sdst[L::kPerThread];   // in buffer 0; buffer 1 lies kBuf elements further
  constexpr int kBuf = L::kBufElems;
#pragma unroll
  for (int i = 0; i < L::kPerThread; ++i) {
    const int p = min((int)threadIdx.x + i * 64 * kOpWaves, npieces - 1);
    const int col = p / L::kPieces, q = p % L::kPieces;
    soff_w[i] = (uint32_t)(((cf0 * 16 + col) * np + q * L::kPer16) * sizeof(VT));
    sdst[i] = &lds[L::off(col, q * L::kPer16)];
  }

  frf a[kRingA][KS];
  piece_t stg[L::kPerThread];
  // TR: row dl of the task's transposed block; rows past N_t hold zeros there
  const rsrc_t rT = TR ? make_rsrc(phiT + (w_off[t] / Rp) * (int64_t)D,
                                   (uint32_t)((int64_t)np * D * 4))
                       : make_rsrc(phi, 0u);   // unused
  const uint32_t aoffT = (uint32_t)(((int64_t)(dl < D ? dl : 0) * np + KS * g4) * 4);
  auto load_a = [&](frf (&x)[KS], int c) __attribute__((always_inline)) {
    const int nb = uniform(min(c, nch - 1) * KC);
    if constexpr (TR) {
      const f4 v = buf_load<f4>(rT, aoffT, (uint32_t)(nb * 4));
#pragma unroll
      for (int s = 0; s < KS; ++s) x[s] = v[s];
    } else {
      const rsrc_t ra = make_rsrc(phit + (int64_t)nb * D,
                                  (uint32_t)((int64_t)max(nt - nb, 0) * D * 4));
#pragma unroll
      for (int s = 0; s < KS; ++s) x[s] = buf_load<frf>(ra, aoff0, (uint32_t)(s * D * 4));
    }
  };
  auto stage_load = [&](int c) __attribute__((always_inline)) {
    const uint32_t soff = (uint32_t)uniform(min(c, nch - 1) * KC * (int)sizeof(VT));
#pragma unroll
    for (int i = 0; i < L::kPerThread; ++i) stg[i] = buf_load<piece_t>(rw, soff_w[i], soff);
  };
  auto stage_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < L::kPerThread; ++i) *(piece_t*)(sdst[i] + buf * kBuf) = stg[i];
  };
  // the W fragments are read in two halves (k-steps 0-1, then 2-3), which halves the registers
  // they hold; the products run in the same order as in k_phit_w
  typedef typename VecOf<VT, 2>::type vt2;
  // nw: the last fragment is narrow (as in k_phi_v_lds)
  auto step = [&](const frf (&x)[KS], int buf, auto nf, auto nw, auto first)
      __attribute__((always_inline)) {
    constexpr int NF = decltype(nf)::value;
    constexpr bool kNw = decltype(nw)::value;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      vt2 b[kColGroup];
#pragma unroll
      for (int cf = 0; cf < kColGroup; ++cf)
        if (cf < NF)
          b[cf] = *(const vt2*)&lds[buf * L::kBufElems +
                                    L::off(cf * 16 + ((kNw && cf == NF - 1) ? (i16 & 3) : i16),
                                           4 * g4 + 2 * h)];
#pragma unroll
      for (int ss = 0; ss < 2; ++ss) {
        const int s = 2 * h + ss;
#pragma unroll
        for (int cf = 0; cf < kColGroup; ++cf)
          if (cf < NF) {
            if constexpr (kNw) {
              if (cf == NF - 1) {
                float av;
                if constexpr (RF == 1) av = x[s]; else av = x[s][0];
                acc4 = mma4<VT>((VT)av, b[cf][ss],
                                (decltype(first)::value && s == 0) ? (VT)0 : acc4);
                continue;
              }
            }
#pragma unroll
            for (int f = 0; f < RF; ++f) {
              float av;
              if constexpr (RF == 1) av = x[s]; else av = x[s][f];
              const acc_t cin = (decltype(first)::value && s == 0) ? acc_t{0, 0, 0, 0} : acc[f][cf];
              acc[f][cf] = Mfma<VT>::mma((VT)av, b[cf][ss], cin);
            }
          }
      }
    }
  };
  // per chunk as in k_phi_v_lds
  auto chunk = [&](int c, auto ic, auto nf, auto nw, auto first) __attribute__((always_inline)) {
    constexpr int i = decltype(ic)::value;
    step(a[i], i & 1, nf, nw, first);
    stage_store((i + 1) & 1);
    stage_load(c + i + 2);
    load_a(a[(i + kRingA - 1) % kRingA], c + i + kRingA - 1);
    __syncthreads();
  };
  auto ring = [&](int c, auto nf, auto nw, auto first) __attribute__((always_inline)) {
    static_for<kRingA>([&](auto ic) __attribute__((always_inline)) {
      chunk(c, ic, nf, nw,
            std::integral_constant<bool, decltype(first)::value && decltype(ic)::value == 0>{});
    });
  };
  auto run = [&](auto nf, auto nw) __attribute__((always_inline)) {
    stage_load(0);
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) load_a(a[i], i);
    stage_store(0);
    stage_load(1);
    __syncthreads();
    int c = 0;
    if (nch >= kRingA) {   // kRingA is even: chunk c + i is in buffer i & 1
      ring(0, nf, nw, std::true_type{});
      for (c = kRingA; c + kRingA <= nch; c += kRingA) ring(c, nf, nw, std::false_type{});
    } else {
      zero_acc();
    }
#pragma unroll
    for (int i = 0; i + 1 < kRingA; ++i) {
      if (c + i >= nch) break;
      step(a[i], i & 1, nf, nw, std::false_type{});
      stage_store((i + 1) & 1);
      stage_load(c + i + 2);
      __syncthreads();
    }
  };
  // one instantiation per fragment count (and narrow last fragment), chosen once per tile:
  // guards on a run-time count inside the pipeline cost more than the skipped products save
  static_for<kColGroup>([&](auto i) __attribute__((always_inline)) {
    constexpr int NF = decltype(i)::value + 1;
    if (ncf != NF) return;
    if constexpr (kNarrowOk<VT, RF>) {
      if (narrow) {
        run(std::integral_constant<int, NF>{}, std::true_type{});
        return;
      }
    }
    run(std::integral_constant<int, NF>{}, std::false_type{});
  });

  phit_w_store<VT, RF>(acc, t, d0, cf0, narrow ? ncf - 1 : ncf, i16, g4, D, Rp, AV, V, alpha,
                       colc, beta, map);
  if constexpr (kNarrowOk<VT, RF>) {
    if (narrow) {
      // bare product (alpha is null here): one value per lane, row narrow_row, column i16 & 3
      const int d = d0 + narrow_row(i16, g4);
      const int slot = map[(ncf - 1) * 16 + (i16 & 3)];
      if (d < D) AV[((int64_t)t * Rp + slot) * D + d] = acc4;
    }
  }
}

template <typename VT, int RF>
static hipError_t phi_v_rf(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                           const VT* V, VT* W, const int* act, const uint8_t* state,
                           hipStream_t st) {
  if constexpr (sizeof(VT) == 4) {
    if (g.fwd_split == kOpWaves) {   // one tile per block
      hipLaunchKernelGGL((k_phi_v<VT, RF, kOpWaves>), dim3(ntiles), dim3(64 * kOpWaves), 0, st,
                         phi, g.row_off, g.w_off, tiles, ntiles, V, W, act, state, g.D, g.Rp);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_phi_v<VT, RF>), dim3((ntiles + kOpWaves - 1) / kOpWaves), dim3(64 * kOpWaves), 0, st, phi,
                     g.row_off, g.w_off, tiles, ntiles, V, W, act, state, g.D, g.Rp);
  return hipGetLastError();
}

template <typename VT, int RF>
static hipError_t phit_w_rf(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                            const VT* W, const VT* V, VT* AV, const float* alpha,
                            const int* colc, double beta, const int* act,
                            const uint8_t* state, hipStream_t st) {
  hipLaunchKernelGGL((k_phit_w<VT, RF>), dim3((ntiles + kOpWaves - 1) / kOpWaves), dim3(64 * kOpWaves), 0, st, phi,
                     g.row_off, g.w_off, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                     g.D, g.Rp);
  return hipGetLastError();
}

template <typename VT, int RF>
static hipError_t phi_v_lds_rf(const Geometry& g, const float* phi, const int4* tiles,
                               int ntiles, const VT* V, VT* W, const int* act, const uint8_t* state,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_phi_v_lds<VT, RF>), dim3(ntiles), dim3(64 * kOpWaves), 0, st, phi,
                     g.row_off, g.w_off, tiles, ntiles, V, W, act, state, g.D, g.Rp);
  return hipGetLastError();
}

template <typename VT, int RF>
static hipError_t phit_w_lds_rf(const Geometry& g, const float* phi, const int4* tiles,
                                int ntiles, const VT* W, const VT* V, VT* AV, const float* alpha,
                                const int* colc, double beta, const int* act,
                            const uint8_t* state, hipStream_t st) {
  if constexpr (RF == 1) {
    if (g.phiT != nullptr) {
      hipLaunchKernelGGL((k_phit_w_lds<VT, RF, true>), dim3(ntiles), dim3(64 * kOpWaves), 0, st,
                         phi, g.row_off, g.w_off, tiles, ntiles, W, V, AV, alpha, colc, beta, act,
                         state, g.D, g.Rp, g.phiT);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_phit_w_lds<VT, RF>), dim3(ntiles), dim3(64 * kOpWaves), 0, st, phi,
                     g.row_off, g.w_off, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                     g.D, g.Rp, nullptr);
  return hipGetLastError();
}

// Phi_t transposed into phiT (task t at element D pt_off[t]: D rows of np_t = pt_off[t + 1] -
// pt_off[t] elements, np_t >= N_t, the rows n >= N_t zero).  One block per 64 x 64 tile of
// (n, d), through LDS so that both the reads (along d) and the writes (along n) are coalesced.
__global__ __launch_bounds__(256) void k_transpose_phi(const float* __restrict__ phi,
                                                      const int64_t* __restrict__ row_off,
                                                      const int64_t* __restrict__ pt_off,
                                                      float* __restrict__ phiT, int D) {
  __shared__ float tile[64][65];
  const int t = blockIdx.z;
  const int n0 = blockIdx.y * 64, d0 = blockIdx.x * 64;
  const int64_t np = pt_off[t + 1] - pt_off[t];
  if (n0 >= np) return;   // uniform over the block
  const int64_t nt = row_off[t + 1] - row_off[t];
  const float* src = phi + row_off[t] * (int64_t)D;
  float* dst = phiT + pt_off[t] * (int64_t)D;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
  for (int i = ty; i < 64; i += 4) {
    const int n = n0 + i, d = d0 + tx;
    tile[i][tx] = (n < nt && d < D) ? src[(int64_t)n * D + d] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int d = d0 + i, n = n0 + tx;
    if (d < D && n < np) dst[(int64_t)d * np + n] = tile[tx][i];
  }
}

hipError_t launch_transpose_phi(const float* phi, const int64_t* row_off, const int64_t* pt_off,
                                float* phiT, int T, int D, int max_np, hipStream_t st) {
  if (T == 0 || max_np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_phi, dim3((D + 63) / 64, (max_np + 63) / 64, T), dim3(256), 0,
                     st, phi, row_off, pt_off, phiT, D);
  return hipGetLastError();
}

template <typename VT>
hipError_t launch_phi_v(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                        const VT* V, VT* W, const int* act, const uint8_t* state, int rows,
                        hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  if (rows < 0) {   // LDS-staged variant: one tile per block of four waves of -rows rows each
    if constexpr (sizeof(VT) == 8) {
      if (rows == -16) return phi_v_lds_rf<VT, 1>(g, phi, tiles, ntiles, V, W, act, state, st);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (sizeof(VT) == 8) {
    if (rows == 16) return phi_v_rf<VT, 1>(g, phi, tiles, ntiles, V, W, act, state, st);
    if (rows == 32) return phi_v_rf<VT, 2>(g, phi, tiles, ntiles, V, W, act, state, st);
  } else {
    if (rows == 16) return phi_v_rf<VT, 1>(g, phi, tiles, ntiles, V, W, act, state, st);
    if (rows == 32) return phi_v_rf<VT, 2>(g, phi, tiles, ntiles, V, W, act, state, st);
    if (rows == 64) return phi_v_rf<VT, 4>(g, phi, tiles, ntiles, V, W, act, state, st);
  }
  return hipErrorInvalidValue;
}

template <typename VT>
hipError_t launch_phit_w(const Geometry& g, const float* phi, const int4* tiles, int ntiles,
                         const VT* W, const VT* V, VT* AV, const float* alpha, const int* colc,
                         double beta, const int* act, const uint8_t* state, int rows,
                         hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  if (rows < 0) {   // LDS-staged variant: one tile per block of four waves of -rows rows each
    if constexpr (sizeof(VT) == 8) {
      if (rows == -16)
        return phit_w_lds_rf<VT, 1>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
    } else {
      if (rows == -32)
        return phit_w_lds_rf<VT, 2>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (sizeof(VT) == 8) {
    if (rows == 16)
      return phit_w_rf<VT, 1>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
    if (rows == 32)
      return phit_w_rf<VT, 2>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
  } else {
    if (rows == 32)
      return phit_w_rf<VT, 2>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
    if (rows == 64)
      return phit_w_rf<VT, 4>(g, phi, tiles, ntiles, W, V, AV, alpha, colc, beta, act, state,
                                     st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_phi_v<double>(const Geometry&, const float*, const int4*, int,
                                         const double*, double*, const int*, const uint8_t*, int,
                                         hipStream_t);
template hipError_t launch_phi_v<float>(const Geometry&, const float*, const int4*, int,
                                        const float*, float*, const int*, const uint8_t*, int,
                                        hipStream_t);
template hipError_t launch_phit_w<double>(const Geometry&, const float*, const int4*, int,
                                          const double*, const double*, double*, const float*,
                                          const int*, double, const int*, const uint8_t*, int,
                                          hipStream_t);
template hipError_t launch_phit_w<float>(const Geometry&, const float*, const int4*, int,
                                         const float*, const float*, float*, const float*,
                                         const int*, double, const int*, const uint8_t*, int,
                                          hipStream_t);

}  // namespace cmtcs
