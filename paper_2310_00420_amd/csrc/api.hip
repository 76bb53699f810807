// C ABI of the library (include/cmtcs.h): handle and workspace management, argument checks,
// and the host loop that drives one batched CG solve (Alg. 1 over all right-hand sides of all
// tasks, Sec. 3.3) per E-step of Alg. 2.
#include <algorithm>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "../../include/cmtcs.h"

using namespace cmtcs;

namespace {

thread_local std::string g_err;

cmtcs_status_t fail(cmtcs_status_t st, const std::string& msg) {
  g_err = msg;
  return st;
}

cmtcs_status_t hip_fail(hipError_t e, const char* what) {
  return fail(CMTCS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, what);     \
  } while (0)

int round16(int x) { return (x + 15) / 16 * 16; }

// An enum field of a caller's struct read as its 32-bit integer.  A caller across the C ABI can
// store any value there, and loading one outside the enumerators as the enum type is undefined
// in C++, so the fields are copied out as integers and checked before use.
template <typename E>
int32_t enum_bits(const E& e) {
  static_assert(sizeof(E) == sizeof(int32_t), "C enums are int-sized here");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

// Task order for a tile table in which every task has the same number of tiles and each tile
// of task t does work w[t] (the adjoint products: a tile contracts over the task's N_t rows).
// Blocks go to the 8 XCDs round-robin and xcd_block gives each XCD a contiguous eighth of the
// table, so the table is laid out as 8 runs of T/8 tasks with nearly equal total work: tasks
// by decreasing work, each onto the least-loaded run that has room; each run then holds its
// tasks longest first.  Tiles of one task stay adjacent (they share the task's W through L2).
std::vector<int> balanced_task_order(const std::vector<int64_t>& w) {
  const int T = (int)w.size();
  std::vector<int> idx(T);
  for (int t = 0; t < T; ++t) idx[t] = t;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] > w[b]; });
  std::vector<std::vector<int>> runs(8);
  std::vector<int64_t> load(8, 0);
  for (int t : idx) {
    int best = -1;
    for (int x = 0; x < 8; ++x) {
      const int cap = T / 8 + (x < T % 8 ? 1 : 0);
      if ((int)runs[x].size() < cap && (best < 0 || load[x] < load[best])) best = x;
    }
    runs[best].push_back(t);
    load[best] += w[t];
  }
  std::vector<int> order;
  order.reserve(T);
  for (const auto& r : runs) order.insert(order.end(), r.begin(), r.end());
  return order;
}

// Profiled steps whose HIP events are harvested together (cmtcs_profile).
constexpr int kCheckEvery = 8;

}  // namespace

struct cmtcs_handle_s {
  int T = 0, C = 0, D = 0;
  double beta = 0.0;
  cmtcs_math_t math = CMTCS_MATH_F64;
  // partial-Fourier sensing: frequencies, multiplier counts m_k + m_{-k} per task, and a
  // counter of out-of-range frequencies found at create
  bool fourier = false;
  const int* freq = nullptr;
  int* hcount = nullptr;
  int* bad_freq = nullptr;
  // Jacobi preconditioner (opts.precond): beta diag(Phi_t^T Phi_t) per task (once), and per call
  // M = diag(A_tc) with sum_d log M; pc_on is set by each entry point for its own launches
  double* mbase = nullptr;
  double* mdiag = nullptr;
  double* slogm = nullptr;
  bool pc_on = false;
  int max_rhs = 0, max_iters = 0, max_K = 0, Rp_max = 0;
  size_t vbytes = 8;
  std::vector<int64_t> row_off;
  int64_t np16 = 0;   // sum over tasks of ceil(N_t / 16)
  // FP64 problems: Phi transposed per task for the LDS-staged adjoint product, rebuilt from Phi
  // at the start of every call that multiplies (so that a caller may change Phi in place)
  float* phiT = nullptr;
  int64_t* pt_off_d = nullptr;
  std::vector<int64_t> pt_off;   // [T + 1]: sum over earlier tasks of N_t rounded up to 16
  int max_np = 0;
  const float* phi = nullptr;
  const float* phi_res = nullptr;   // MATH_MIXED: Phi of the FP32 true-residual products
  const float* y = nullptr;
  hipStream_t st = nullptr;

  std::vector<void*> allocs;
  int64_t* row_off_d = nullptr;
  int64_t* w_off_d = nullptr;
  double* lconst = nullptr;   // [T] constant of each task's marginal log-likelihood
  void *X = nullptr, *Rv = nullptr, *Dv = nullptr, *AD = nullptr, *W = nullptr, *b = nullptr;
  double *rr = nullptr, *thr = nullptr, *gam = nullptr, *xi = nullptr;
  uint8_t* state = nullptr;
  bool compact = true;
  int* iters = nullptr;
  int* act = nullptr;
  int* colc = nullptr;
  int4* fwd_tiles = nullptr;
  int4* adj_tiles = nullptr;
  int nfwd = 0, nadj = 0, cur_Rp = -1;
  // output rows per wave tile of the two products (autotuned per column count)
  int fwd_rows = 0, adj_rows = 0, cur_fwd_rows = -1, cur_adj_rows = -1, tuned_Rp = -1;
  bool autotune = true;
  void* slq_ws = nullptr;
  long slq_lds = kSlqLdsBytes;   // LDS budget of the SLQ kernel (CMTCS_SLQ_LDS_BYTES)
  double *tau = nullptr, *rmin = nullptr,
         *rmax = nullptr, *slog = nullptr;
  uint8_t* ok = nullptr;
  int* keff = nullptr;       // [T][C] probes that entered nu-bar
  int* act_host = nullptr;   // pinned; read while profiling only

  // mixed precision (CMTCS_MATH_MIXED)
  void* phi16 = nullptr;                 // 16-bit copy of Phi, [rows][D]
  cmtcs_dtype_t phi_dtype = CMTCS_F32;
  void* phiT16 = nullptr;                // [D][np32_t] per task
  void* D16 = nullptr;                   // 16-bit copy of the CG direction
  void* W16 = nullptr;                   // [Rp][np32_t] per task
  int64_t* w16_off_d = nullptr;
  int4* fwd16_tiles = nullptr;
  int4* adj16_tiles = nullptr;
  int nfwd16 = 0, nadj16 = 0, max_np32 = 0;

  // recorded CG loop (opts.graph)
  hipStream_t cap_st = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  struct GraphKey {
    const float* alpha; int R, Rp, steps, fixed, fwd_rows, adj_rows; bool pc;
    bool operator==(const GraphKey& o) const {
      return alpha == o.alpha && R == o.R && Rp == o.Rp && steps == o.steps && fixed == o.fixed &&
             fwd_rows == o.fwd_rows && adj_rows == o.adj_rows && pc == o.pc;
    }
  } graph_key{};
  // recorded EM iteration (cmtcs_em_iter with opts.graph): E-step and M-step as one graph
  hipGraph_t em_graph = nullptr;
  hipGraphExec_t em_exec = nullptr;
  struct EmKey {
    const void* p[8];   // alpha, log_pi, mu, s, logdet, ell, q, probes
    int K, steps, fixed, R, Rp, fwd_rows, adj_rows, crn, pc;
    double tol, alpha_max;
    bool operator==(const EmKey& o) const {
      for (int i = 0; i < 8; ++i)
        if (p[i] != o.p[i]) return false;
      return K == o.K && steps == o.steps && fixed == o.fixed && R == o.R && Rp == o.Rp &&
             fwd_rows == o.fwd_rows && adj_rows == o.adj_rows && crn == o.crn && pc == o.pc &&
             tol == o.tol && alpha_max == o.alpha_max;
    }
  } em_key{};
  // probe key of the current E-step, read by the kernels that draw probes (a device word, so
  // that a recorded E-step replays with the key of each new EM iteration)
  uint64_t* key_d = nullptr;

  // kernel timing (cmtcs_profile)
  bool prof_on = false;
  hipEvent_t ev[kCheckEvery][4] = {};
  bool ev_made = false;
  int ev_pending = 0;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};

  template <typename P>
  hipError_t alloc(P** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = (P*)q;
    return hipSuccess;
  }

  ~cmtcs_handle_s() {
    for (void* p : allocs) (void)hipFree(p);
    if (act_host) (void)hipHostFree(act_host);
    if (ev_made)
      for (auto& row : ev)
        for (auto& e : row) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (em_exec) (void)hipGraphExecDestroy(em_exec);
    if (em_graph) (void)hipGraphDestroy(em_graph);
    if (cap_st) (void)hipStreamDestroy(cap_st);
  }

  // Records the `steps` CG steps of run_cg as one graph (on a private stream: the caller's
  // stream may be the null stream, which cannot be captured) and launches it on the handle's
  // stream; the recording is reused while its key matches.
  template <typename VT>
  cmtcs_status_t run_cg_graph(const Geometry& g, const float* alpha, int steps, int fixed) {
    const GraphKey key{alpha, g.R, g.Rp, steps, fixed, fwd_rows, adj_rows, pc_on};
    if (graph_exec == nullptr || !(key == graph_key)) {
      if (graph_exec) { (void)hipGraphExecDestroy(graph_exec); graph_exec = nullptr; }
      if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
      if (cap_st == nullptr)
        HIP_TRY(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking), "hipStreamCreate");
      HIP_TRY(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed),
              "hipStreamBeginCapture");
      hipError_t e = cg_steps_all<VT>(g, alpha, steps, fixed, cap_st);
      hipGraph_t gr = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cap_st, &gr);
      if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(e, "graph recording");
      }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      graph = gr;
      HIP_TRY(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0),
              "hipGraphInstantiate");
      graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(graph_exec, st), "hipGraphLaunch");
    return CMTCS_OK;
  }

  // All `steps` CG steps (three launches each) on stream s, with no host check in between:
  // columns and tasks that have stopped return at once inside the kernels.  The form a graph
  // records.
  template <typename VT>
  hipError_t cg_steps_all(const Geometry& g, const float* alpha, int steps, int fixed,
                          hipStream_t s) {
    const CgState cs = cg_loop(alpha);
    hipError_t e = hipSuccess;
    for (int u = 0; u < steps && e == hipSuccess; ++u) {
      const int* act_u = act + (size_t)u * T;
      e = launch_phi_v<VT>(g, phi, fwd_tiles, nfwd, (const VT*)Dv, (VT*)W, act_u, cstate(),
                           fwd_rows, s);
      if (e == hipSuccess)
        e = launch_phit_w<VT>(g, phi, adj_tiles, nadj, (const VT*)W, (const VT*)Dv, (VT*)AD,
                              nullptr, colc, beta, act_u, cstate(), adj_rows, s);
      if (e == hipSuccess) e = launch_cg_update<VT>(g, cs, u, steps, fixed, 0, s);
    }
    return e;
  }

  // Adds the durations of the `ev_pending` timed steps recorded so far.
  hipError_t harvest() {
    for (int i = 0; i < ev_pending; ++i) {
      hipError_t e = hipEventSynchronize(ev[i][3]);
      if (e != hipSuccess) return e;
      for (int k = 0; k < 3; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i][k], ev[i][k + 1]);
        if (e != hipSuccess) return e;
        prof_ms[k] += ms;
        prof_n[k] += 1;
      }
    }
    ev_pending = 0;
    return hipSuccess;
  }

  Geometry geom(int R, int Rp) const {
    Geometry g;
    g.T = T; g.C = C; g.D = D; g.R = R; g.Rp = Rp;
    g.row_off = row_off_d; g.w_off = w_off_d;
    g.fwd_split = fwd_split_of(np16, Rp, D);
    g.phiT = phiT;
    return g;
  }

  // Geometry of an operator call, with phiT rebuilt from Phi first
  cmtcs_status_t op_geom(int R, int Rp, Geometry* g) {
    *g = geom(R, Rp);
    if (phiT != nullptr)
      HIP_TRY(launch_transpose_phi(phi, row_off_d, pt_off_d, phiT, T, D, max_np, st),
              "launch(transpose_phi)");
    return CMTCS_OK;
  }

  Geometry geom16(int R, int Rp) const {
    Geometry g = geom(R, Rp);
    g.w_off = w16_off_d;
    return g;
  }

  bool mixed() const { return math == CMTCS_MATH_MIXED; }

  // The whole CG solve of a partial-Fourier problem: one kernel (timed in the third profiling
  // slot while profiling is on).
  cmtcs_status_t run_fourier(const Geometry& g, const float* alpha, int mode,
                             const RhsSource& src, double tol, int steps, int fixed) {
    const CgState s = cg_loop(alpha);
    hipEvent_t* e4 = prof_on ? ev[ev_pending] : nullptr;
    if (e4) {
      for (int k = 0; k < 3; ++k) HIP_TRY(hipEventRecord(e4[k], st), "hipEventRecord");
    }
    HIP_TRY(launch_fourier_cg(g, s, hcount, mode, src, tol, steps, fixed, st),
            "launch(fourier_cg)");
    if (e4) {
      HIP_TRY(hipEventRecord(e4[3], st), "hipEventRecord");
      if (++ev_pending == kCheckEvery) HIP_TRY(harvest(), "profile events");
    }
    return CMTCS_OK;
  }

  // Column states for the products of the CG loop (compaction of active columns), unless
  // CMTCS_COMPACT=0 was set at create.
  const uint8_t* cstate() const { return compact ? state : nullptr; }

  CgState cg() const {
    CgState s;
    s.X = X; s.Rv = Rv; s.Dv = Dv; s.AD = AD;
    s.rr = rr; s.thr = thr; s.state = state; s.iters = iters;
    s.gam = gam; s.xi = xi; s.act = act;
    s.alpha = nullptr; s.colc = colc; s.beta = beta;
    s.d16 = nullptr; s.d16_kind = 0; s.d16_ld = 0;
    s.mdiag = pc_on ? mdiag : nullptr;
    return s;
  }

  // State for the CG loop: the adjoint product (FP64, FP32 or 16-bit) stores the bare
  // Phi^T Phi d and the update adds beta and the diagonal term.
  CgState cg_loop(const float* alpha) const {
    CgState s = cg();
    s.alpha = alpha;
    return s;
  }

  int ngroups(int Rp) const { return Rp / 16 / group_width(Rp); }

  // Tile tables and W offsets for Rp column slots per task (rebuilt only when Rp changes).
  cmtcs_status_t prepare(int Rp) {
    if (Rp == cur_Rp && fwd_rows == cur_fwd_rows && adj_rows == cur_adj_rows) return CMTCS_OK;
    const int fr = fwd_rows, ar = adj_rows, ng = ngroups(Rp);
    std::vector<int64_t> woff(T + 1, 0), adj_work(T);
    std::vector<int4> ft, at;
    for (int t = 0; t < T; ++t) {
      const int nt = (int)(row_off[t + 1] - row_off[t]);
      const int np = round16(nt);
      woff[t + 1] = woff[t] + (int64_t)Rp * np;
      // forward tiles: the same work each (a contraction over D), so equal counts per XCD
      // balance them in task order
      for (int n0 = 0; n0 < np; n0 += tile_step(fr))
        for (int cg = 0; cg < ng; ++cg) ft.push_back(make_int4(t, n0, cg, 0));
      adj_work[t] = np + 16;   // contraction rows, plus the epilogue as a few more
    }
    for (int t : balanced_task_order(adj_work))
      for (int d0 = 0; d0 < D; d0 += tile_step(ar))
        for (int cg = 0; cg < ng; ++cg) at.push_back(make_int4(t, d0, cg, 0));
    HIP_TRY(hipMemcpyAsync(w_off_d, woff.data(), sizeof(int64_t) * (T + 1),
                           hipMemcpyHostToDevice, st), "hipMemcpyAsync(w_off)");
    if (!ft.empty())
      HIP_TRY(hipMemcpyAsync(fwd_tiles, ft.data(), sizeof(int4) * ft.size(),
                             hipMemcpyHostToDevice, st), "hipMemcpyAsync(fwd tiles)");
    HIP_TRY(hipMemcpyAsync(adj_tiles, at.data(), sizeof(int4) * at.size(),
                           hipMemcpyHostToDevice, st), "hipMemcpyAsync(adj tiles)");
    if (mixed()) {
      std::vector<int64_t> w16(T + 1, 0), adj16_work(T);
      std::vector<int4> f16, a16;
      for (int t = 0; t < T; ++t) {
        const int np = (int)((row_off[t + 1] - row_off[t] + 31) / 32 * 32);
        w16[t + 1] = w16[t] + (int64_t)Rp * ld16(np);
        for (int n0 = 0; n0 < np; n0 += 4 * kRows16)   // one tile per block of four waves
          for (int cg = 0; cg < ng; ++cg) f16.push_back(make_int4(t, n0, cg, 0));
        adj16_work[t] = np + 32;
      }
      for (int t : balanced_task_order(adj16_work))
        for (int d0 = 0; d0 < D; d0 += 4 * kRows16)
          for (int cg = 0; cg < ng; ++cg) a16.push_back(make_int4(t, d0, cg, 0));
      HIP_TRY(hipMemcpyAsync(w16_off_d, w16.data(), sizeof(int64_t) * (T + 1),
                             hipMemcpyHostToDevice, st), "hipMemcpyAsync(w16_off)");
      if (!f16.empty())
        HIP_TRY(hipMemcpyAsync(fwd16_tiles, f16.data(), sizeof(int4) * f16.size(),
                               hipMemcpyHostToDevice, st), "hipMemcpyAsync(fwd16 tiles)");
      HIP_TRY(hipMemcpyAsync(adj16_tiles, a16.data(), sizeof(int4) * a16.size(),
                             hipMemcpyHostToDevice, st), "hipMemcpyAsync(adj16 tiles)");
      HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(prepare16)");
      nfwd16 = (int)f16.size();
      nadj16 = (int)a16.size();
    }
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(prepare)");
    nfwd = (int)ft.size();
    nadj = (int)at.size();
    cur_Rp = Rp;
    cur_fwd_rows = fwd_rows;
    cur_adj_rows = adj_rows;
    return CMTCS_OK;
  }

  // Autotuner: for a new column count, times every supported tile shape of each product on
  // the handle's own buffers (one warm-up and three timed launches, HIP events on the
  // handle's stream, each after a launch of the other product) and keeps the fastest.  Runs before the solve initialises its vectors;
  // the products only read the workspace and write W and AD.
  template <typename VT>
  cmtcs_status_t tune(const Geometry& g, const float* alpha) {
    if (!autotune || mixed() || tuned_Rp == g.Rp) return prepare(g.Rp);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    cmtcs_status_t rs = CMTCS_OK;
    for (int kind = 0; kind < 2 && rs == CMTCS_OK; ++kind) {
      int cand[kMaxTileCands];
      const int nc = op_row_candidates(math == CMTCS_MATH_F64, kind, cand);
      float best = 1e30f;
      int best_rows = kind == 0 ? fwd_rows : adj_rows;
      for (int i = 0; i < nc && rs == CMTCS_OK; ++i) {
        (kind == 0 ? fwd_rows : adj_rows) = cand[i];
        rs = prepare(g.Rp);
        if (rs != CMTCS_OK) break;
        // each timed launch follows a launch of the other product, as in a CG step, so that
        // the candidate meets the cache state the loop leaves (its own operands evicted)
        float ms = 0.f;
        hipError_t e = hipSuccess;
        auto fwd = [&]() {
          return launch_phi_v<VT>(g, phi, fwd_tiles, nfwd, (const VT*)Dv, (VT*)W, nullptr,
                                  nullptr, fwd_rows, st);
        };
        auto adj = [&]() {
          return launch_phit_w<VT>(g, phi, adj_tiles, nadj, (const VT*)W, (const VT*)Dv,
                                   (VT*)AD, nullptr, colc, beta, nullptr, nullptr, adj_rows,
                                   st);
        };
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
          e = kind == 0 ? adj() : fwd();
          if (e == hipSuccess) e = hipEventRecord(e0, st);
          if (e == hipSuccess) e = kind == 0 ? fwd() : adj();
          if (e == hipSuccess) e = hipEventRecord(e1, st);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float one = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&one, e0, e1);
          if (rep > 0) ms += one;   // the first round is a warm-up
        }
        if (e != hipSuccess) { rs = hip_fail(e, "autotune"); break; }
        if (ms < best) { best = ms; best_rows = cand[i]; }
      }
      (kind == 0 ? fwd_rows : adj_rows) = best_rows;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != CMTCS_OK) return rs;
    tuned_Rp = g.Rp;
    return prepare(g.Rp);
  }

  // 16-bit products of one step (MATH_MIXED); which = 1: Phi V16, 2: Phi^T W16 (+ beta and
  // alpha V when alpha is given; the CG loop passes none and the update adds them).
  hipError_t mixed_product(const Geometry& g16, const float* alpha, const int* act_u,
                           int which) {
    if (phi_dtype == CMTCS_BF16)
      return launch_mixed_products<__bf16>(g16, phi16, phiT16, fwd16_tiles, nfwd16, adj16_tiles,
                                           nadj16, D16, W16, (const float*)Dv, (float*)AD,
                                           alpha, colc, beta, act_u, which, st);
    return launch_mixed_products<_Float16>(g16, phi16, phiT16, fwd16_tiles, nfwd16, adj16_tiles,
                                           nadj16, D16, W16, (const float*)Dv, (float*)AD,
                                           alpha, colc, beta, act_u, which, st);
  }

  hipError_t round_direction(const Geometry& g) {
    const int64_t rows = (int64_t)T * g.Rp;
    if (phi_dtype == CMTCS_BF16)
      return launch_round16<__bf16>((const float*)Dv, D, D16, ld16(D), rows, D, st);
    return launch_round16<_Float16>((const float*)Dv, D, D16, ld16(D), rows, D, st);
  }

  // Enqueues all `steps` CG steps without waiting: the kernels of a step return at once for
  // tasks (products) and columns (update) that have stopped.
  template <typename VT>
  cmtcs_status_t run_cg(const Geometry& g, const float* alpha, int steps, int fixed,
                        const RhsSource& src, int refine_every) {
    CgState s = cg_loop(alpha);
    if (mixed()) {
      s.d16 = D16;
      s.d16_kind = phi_dtype == CMTCS_BF16 ? 1 : 2;
      s.d16_ld = ld16(D);
    }
    const Geometry g16 = geom16(g.R, g.Rp);
    if (mixed()) HIP_TRY(round_direction(g), "launch(round16)");
    for (int u = 0; u < steps; ++u) {
      const int* act_u = act + (size_t)u * T;
      hipEvent_t* e4 = prof_on ? ev[ev_pending] : nullptr;
      if (e4) HIP_TRY(hipEventRecord(e4[0], st), "hipEventRecord");
      if (mixed())
        HIP_TRY(mixed_product(g16, alpha, act_u, 1), "launch(phi_v16)");
      else
        HIP_TRY(launch_phi_v<VT>(g, phi, fwd_tiles, nfwd, (const VT*)Dv, (VT*)W, act_u,
                                  cstate(), fwd_rows, st),
                "launch(phi_v)");
      if (e4) HIP_TRY(hipEventRecord(e4[1], st), "hipEventRecord");
      if (mixed())
        HIP_TRY(mixed_product(g16, nullptr, act_u, 2), "launch(phit_w16)");
      else
        HIP_TRY(launch_phit_w<VT>(g, phi, adj_tiles, nadj, (const VT*)W, (const VT*)Dv,
                                  (VT*)AD, nullptr, colc, beta, act_u, cstate(), adj_rows, st),
                "launch(phit_w)");
      if (e4) HIP_TRY(hipEventRecord(e4[2], st), "hipEventRecord");
      const bool replace = mixed() && refine_every > 0 && (u + 1) % refine_every == 0;
      HIP_TRY(launch_cg_update<VT>(g, s, u, steps, fixed, replace ? 1 : 0, st),
              "launch(cg_update)");
      if (replace) {
        // true-residual replacement: r = b - A x with FP32 products from the FP32 Phi, then
        // xi, d and the stop decision from the replaced residual
        HIP_TRY(launch_phi_v<float>(g, phi_res, fwd_tiles, nfwd, (const float*)X, (float*)W,
                                    act_u, nullptr, fwd_rows, st), "launch(phi_v residual)");
        HIP_TRY(launch_phit_w<float>(g, phi_res, adj_tiles, nadj, (const float*)W, (const float*)X,
                                     (float*)AD, alpha, colc, beta, act_u, nullptr, adj_rows,
                                     st),
                "launch(phit_w residual)");
        HIP_TRY(launch_replace(g, s, (const float*)AD, src, u, steps, fixed, st),
                "launch(replace)");
      }
      // the update wrote the 16-bit direction itself, except on replacement steps
      if (replace) HIP_TRY(round_direction(g), "launch(round16)");
      if (e4) {
        HIP_TRY(hipEventRecord(e4[3], st), "hipEventRecord");
        if (++ev_pending == kCheckEvery) {
          // while profiling, the host waits here for the timings anyway; it also reads the
          // active counts and stops enqueueing once every column has stopped, so that the
          // timings hold the steps that did work and not the trailing empty launches
          HIP_TRY(harvest(), "profile events");
          if (u + 1 < steps) {
            HIP_TRY(hipMemcpyAsync(act_host, act + (size_t)(u + 1) * T, sizeof(int) * T,
                                   hipMemcpyDeviceToHost, st), "hipMemcpyAsync(active counts)");
            HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(active counts)");
            bool any = false;
            for (int t = 0; t < T; ++t) any = any || act_host[t] != 0;
            if (!any) break;
          }
        }
      }
    }
    if (prof_on) HIP_TRY(harvest(), "profile events");
    return CMTCS_OK;
  }

  template <typename VT>
  cmtcs_status_t apply(const float* alpha, int R, const int32_t* col_cluster, const void* V,
                       void* AV) {
    pc_on = false;
    const int Rp = col_slots(R);
    if (fourier) {
      const Geometry g = geom(R, Rp);
      HIP_TRY(launch_fill_colc(colc, T, R, Rp, 0, col_cluster, st), "launch(fill_colc)");
      RhsSource src;
      src.kind = 1; src.b = nullptr; src.B = V; src.K = 0; src.keyp = nullptr;
      src.probes = nullptr; src.crn = 0;
      cmtcs_status_t rs = run_fourier(g, alpha, 1, src, 0.0, 0, 1);
      if (rs != CMTCS_OK) return rs;
      HIP_TRY(launch_solve_output<VT>(g, cg(), AV, nullptr, nullptr, 0, nullptr, nullptr, st),
              "launch(copy out)");
      return CMTCS_OK;
    }
    cmtcs_status_t rs = prepare(Rp);
    if (rs != CMTCS_OK) return rs;
    Geometry g;
    rs = op_geom(R, Rp, &g);
    if (rs != CMTCS_OK) return rs;
    HIP_TRY(launch_fill_colc(colc, T, R, Rp, 0, col_cluster, st), "launch(fill_colc)");
    RhsSource src;
    src.kind = 1; src.b = nullptr; src.B = V; src.K = 0; src.keyp = nullptr; src.probes = nullptr;
    src.crn = 0;
    HIP_TRY(launch_cg_init<VT>(g, cg(), src, 0.0, 0, st), "launch(cg_init)");
    HIP_TRY(launch_phi_v<VT>(g, phi, fwd_tiles, nfwd, (const VT*)Dv, (VT*)W, nullptr, nullptr,
                             fwd_rows, st), "launch(phi_v)");
    HIP_TRY(launch_phit_w<VT>(g, phi, adj_tiles, nadj, (const VT*)W, (const VT*)Dv, (VT*)AD,
                              alpha, colc, beta, nullptr, nullptr, adj_rows, st),
            "launch(phit_w)");
    CgState s = cg();
    s.X = AD;   // copy A V out through the solution-copy kernel
    HIP_TRY(launch_solve_output<VT>(g, s, AV, nullptr, nullptr, 0, nullptr, nullptr, st),
            "launch(copy out)");
    return CMTCS_OK;
  }

  template <typename VT>
  cmtcs_status_t grad(int R, const int32_t* col_cluster, const void* Xs, const void* Lam,
                      double y_coef, float* dalpha, float* dphi) {
    pc_on = false;
    const int Rp = col_slots(2 * R);
    cmtcs_status_t rs = prepare(Rp);
    if (rs != CMTCS_OK) return rs;
    const Geometry g = geom(2 * R, Rp);
    HIP_TRY(launch_fill_colc(colc, T, R, Rp, 0, col_cluster, st), "launch(fill_colc)");
    HIP_TRY(launch_pack2<VT>(geom(R, Rp), Xs, Lam, Dv, st), "launch(pack2)");
    HIP_TRY(launch_phi_v<VT>(g, phi, fwd_tiles, nfwd, (const VT*)Dv, (VT*)W, nullptr, nullptr,
                             fwd_rows, st), "launch(phi_v)");
    HIP_TRY(launch_grads<VT>(g, R, (const VT*)Dv, (const VT*)W, y, colc, beta, y_coef, dalpha,
                             dphi, row_off[T], st), "launch(grads)");
    return CMTCS_OK;
  }

  template <typename VT>
  cmtcs_status_t estep(const float* alpha, const double* log_pi, const cmtcs_opts_t& o,
                       float* mu, float* sd, double* logdet, double* ell, double* q,
                       cmtcs_cg_stats_t* stats) {
    const int K = o.K, R = C * (K + 1), Rp = col_slots(R);
    cmtcs_status_t rs = fourier ? CMTCS_OK : prepare(Rp);
    if (rs != CMTCS_OK) return rs;
    Geometry g;
    rs = op_geom(R, Rp, &g);
    if (rs != CMTCS_OK) return rs;
    const uint64_t key = probe_key(o.seed, o.em_iter);
    const int fixed = o.fixed_iters > 0 ? 1 : 0;
    const int steps = fixed ? o.fixed_iters : o.max_iters;
    HIP_TRY(launch_fill_colc(colc, T, R, Rp, K, nullptr, st), "launch(fill_colc)");
    if (!fourier) rs = tune<VT>(g, alpha);
    if (rs != CMTCS_OK) return rs;
    HIP_TRY(launch_set_key(key_d, key, st), "launch(set_key)");
    pc_on = o.precond != 0;
    if (pc_on) HIP_TRY(launch_jacobi(g, mbase, alpha, mdiag, slogm, st), "launch(jacobi)");
    RhsSource src;
    src.kind = 0; src.b = b; src.B = nullptr; src.K = K; src.keyp = key_d; src.probes = o.probes;
    src.crn = o.common_probes;
    if (fourier) {
      rs = run_fourier(g, alpha, 0, src, fixed ? 0.0 : o.tol, steps, fixed);
    } else {
      HIP_TRY(launch_cg_init<VT>(g, cg(), src, fixed ? 0.0 : o.tol, steps, st),
              "launch(cg_init)");
      if (o.graph && !mixed()) rs = run_cg_graph<VT>(g, alpha, steps, fixed);
      else rs = run_cg<VT>(g, alpha, steps, fixed, src, o.refine_every);
    }
    if (rs != CMTCS_OK) return rs;
    HIP_TRY(launch_estep_finalize<VT>(g, cg(), K, key_d, o.probes, o.common_probes, mu, sd, st),
            "launch(estep_finalize)");
    HIP_TRY(launch_sum_log_alpha(C, D, alpha, slog, st), "launch(sum_log_alpha)");
    HIP_TRY(launch_slq(g, cg(), K, steps, (double)D, slq_ws, tau, ok, rmin, rmax, slq_lds, st),
            "launch(slq)");
    HIP_TRY(launch_resp<VT>(g, cg(), K, (const VT*)b, tau, ok, slog, log_pi, logdet, ell, q,
                            keff, pc_on ? slogm : nullptr, st),
            "launch(resp)");
    if (stats != nullptr) {
      HIP_TRY(launch_stats_estep(g, cg(), K, ok, keff, stats->iters, stats->status, stats->k_eff,
                                 st), "launch(stats)");
      const size_t P = (size_t)T * C * K;
      if (stats->ritz_min != nullptr)
        HIP_TRY(hipMemcpyAsync(stats->ritz_min, rmin, sizeof(double) * P,
                               hipMemcpyDeviceToDevice, st), "hipMemcpyAsync(ritz_min)");
      if (stats->ritz_max != nullptr)
        HIP_TRY(hipMemcpyAsync(stats->ritz_max, rmax, sizeof(double) * P,
                               hipMemcpyDeviceToDevice, st), "hipMemcpyAsync(ritz_max)");
    }
    return CMTCS_OK;
  }

  // The device work of one EM iteration (E-step without stats, then the M-step) on stream s,
  // with the fixed-length CG loop: what cmtcs_em_iter records as one graph.
  template <typename VT>
  hipError_t em_launches(const Geometry& g, float* alpha, const double* log_pi,
                         const cmtcs_opts_t& o, int steps, int fixed, float* mu, float* sd,
                         double* logdet, double* ell, double* q, hipStream_t s) {
    const int K = o.K;
    RhsSource src;
    src.kind = 0; src.b = b; src.B = nullptr; src.K = K; src.keyp = key_d; src.probes = o.probes;
    src.crn = o.common_probes;
    // the cluster map is rewritten here (other calls on the handle reuse its buffer)
    hipError_t e = launch_fill_colc(colc, T, g.R, g.Rp, K, nullptr, s);
    if (e == hipSuccess && pc_on) e = launch_jacobi(g, mbase, alpha, mdiag, slogm, s);
    if (e == hipSuccess) e = launch_cg_init<VT>(g, cg(), src, fixed ? 0.0 : o.tol, steps, s);
    if (e == hipSuccess) e = cg_steps_all<VT>(g, alpha, steps, fixed, s);
    if (e == hipSuccess)
      e = launch_estep_finalize<VT>(g, cg(), K, key_d, o.probes, o.common_probes, mu, sd, s);
    if (e == hipSuccess) e = launch_sum_log_alpha(C, D, alpha, slog, s);
    if (e == hipSuccess)
      e = launch_slq(g, cg(), K, steps, (double)D, slq_ws, tau, ok, rmin, rmax, slq_lds, s);
    if (e == hipSuccess)
      e = launch_resp<VT>(g, cg(), K, (const VT*)b, tau, ok, slog, log_pi, logdet, ell, q, keff,
                          pc_on ? slogm : nullptr, s);
    if (e == hipSuccess) e = launch_mstep(T, C, D, mu, sd, q, o.alpha_max, alpha, s);
    return e;
  }

  // One EM iteration (Alg. 2): the E-step from alpha, then the M-step into alpha.  With
  // opts.graph (MATH_F64 / MATH_F32) the whole device sequence is recorded once per shape,
  // step policy and set of buffers and replayed; only the probe key (a device word set before
  // the replay) changes from one iteration to the next.
  template <typename VT>
  cmtcs_status_t em_iter(float* alpha, const double* log_pi, const cmtcs_opts_t& o, float* mu,
                         float* sd, double* logdet, double* ell, double* q) {
    if (!o.graph || mixed() || fourier) {
      cmtcs_status_t rs = estep<VT>(alpha, log_pi, o, mu, sd, logdet, ell, q, nullptr);
      if (rs != CMTCS_OK) return rs;
      HIP_TRY(launch_mstep(T, C, D, mu, sd, q, o.alpha_max, alpha, st), "launch(mstep)");
      return CMTCS_OK;
    }
    const int K = o.K, R = C * (K + 1), Rp = col_slots(R);
    cmtcs_status_t rs = prepare(Rp);
    if (rs != CMTCS_OK) return rs;
    Geometry g;
    rs = op_geom(R, Rp, &g);
    if (rs != CMTCS_OK) return rs;
    const int fixed = o.fixed_iters > 0 ? 1 : 0;
    const int steps = fixed ? o.fixed_iters : o.max_iters;
    HIP_TRY(launch_fill_colc(colc, T, R, Rp, K, nullptr, st), "launch(fill_colc)");
    rs = tune<VT>(g, alpha);   // trial launches happen here, never inside a recording
    if (rs != CMTCS_OK) return rs;
    HIP_TRY(launch_set_key(key_d, probe_key(o.seed, o.em_iter), st), "launch(set_key)");
    pc_on = o.precond != 0;
    const EmKey key{{alpha, log_pi, mu, sd, logdet, ell, q, o.probes}, K, steps, fixed, R, Rp,
                    fwd_rows, adj_rows, o.common_probes, o.precond,
                    fixed ? 0.0 : o.tol, o.alpha_max};
    if (em_exec == nullptr || !(key == em_key)) {
      if (em_exec) { (void)hipGraphExecDestroy(em_exec); em_exec = nullptr; }
      if (em_graph) { (void)hipGraphDestroy(em_graph); em_graph = nullptr; }
      if (cap_st == nullptr)
        HIP_TRY(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking), "hipStreamCreate");
      HIP_TRY(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed),
              "hipStreamBeginCapture");
      const hipError_t e = em_launches<VT>(g, alpha, log_pi, o, steps, fixed, mu, sd, logdet,
                                           ell, q, cap_st);
      hipGraph_t gr = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cap_st, &gr);
      if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(e, "graph recording (EM iteration)");
      }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      em_graph = gr;
      HIP_TRY(hipGraphInstantiate(&em_exec, em_graph, nullptr, nullptr, 0),
              "hipGraphInstantiate");
      em_key = key;
    }
    HIP_TRY(hipGraphLaunch(em_exec, st), "hipGraphLaunch");
    return CMTCS_OK;
  }

  template <typename VT>
  cmtcs_status_t solve(const float* alpha, int R, const int32_t* col_cluster, const void* B,
                       void* Xout, double* gout, double* xout, const cmtcs_opts_t& o,
                       cmtcs_cg_stats_t* stats) {
    const int Rp = col_slots(R);
    cmtcs_status_t rs = fourier ? CMTCS_OK : prepare(Rp);
    if (rs != CMTCS_OK) return rs;
    Geometry g;
    rs = op_geom(R, Rp, &g);
    if (rs != CMTCS_OK) return rs;
    const int fixed = o.fixed_iters > 0 ? 1 : 0;
    const int steps = fixed ? o.fixed_iters : o.max_iters;
    HIP_TRY(launch_fill_colc(colc, T, R, Rp, 0, col_cluster, st), "launch(fill_colc)");
    if (!fourier) rs = tune<VT>(g, alpha);
    if (rs != CMTCS_OK) return rs;
    RhsSource src;
    src.kind = 1; src.b = nullptr; src.B = B; src.K = 0; src.keyp = nullptr; src.probes = nullptr;
    src.crn = 0;
    pc_on = o.precond != 0;
    if (pc_on) HIP_TRY(launch_jacobi(g, mbase, alpha, mdiag, slogm, st), "launch(jacobi)");
    if (fourier) {
      rs = run_fourier(g, alpha, 0, src, fixed ? 0.0 : o.tol, steps, fixed);
    } else {
      HIP_TRY(launch_cg_init<VT>(g, cg(), src, fixed ? 0.0 : o.tol, steps, st),
              "launch(cg_init)");
      if (o.graph && !mixed()) rs = run_cg_graph<VT>(g, alpha, steps, fixed);
      else rs = run_cg<VT>(g, alpha, steps, fixed, src, o.refine_every);
    }
    if (rs != CMTCS_OK) return rs;
    HIP_TRY(launch_solve_output<VT>(g, cg(), Xout, gout, xout, steps,
                                    stats ? stats->iters : nullptr,
                                    stats ? stats->status : nullptr, st),
            "launch(solve_output)");
    return CMTCS_OK;
  }
};

namespace {

cmtcs_status_t check_opts(const cmtcs_handle_s* h, const cmtcs_opts_t* o, bool need_K) {
  if (o == nullptr) return fail(CMTCS_E_INVALID, "opts is NULL");
  if (o->fixed_iters < 0) return fail(CMTCS_E_INVALID, "fixed_iters < 0");
  if (o->fixed_iters > 0) {
    if (o->fixed_iters > h->max_iters)
      return fail(CMTCS_E_INVALID, "fixed_iters exceeds the handle's max_iters");
  } else {
    if (o->max_iters < 1 || o->max_iters > h->max_iters)
      return fail(CMTCS_E_INVALID, "max_iters must be in 1..handle max_iters");
    if (!(o->tol >= 0.0)) return fail(CMTCS_E_INVALID, "tol must be >= 0");
  }
  if (o->common_probes != 0 && o->common_probes != 1)
    return fail(CMTCS_E_INVALID, "common_probes must be 0 or 1");
  if (o->precond != 0 && o->precond != 1) return fail(CMTCS_E_INVALID, "precond must be 0 or 1");
  if (o->precond && (h->math == CMTCS_MATH_MIXED || h->fourier))
    return fail(CMTCS_E_UNSUPPORTED,
                "precond is available for dense problems in MATH_F64 and MATH_F32 only");
  if (need_K) {
    if (o->K < 1 || o->K > h->max_K) return fail(CMTCS_E_INVALID, "K must be in 1..max_K");
    if ((int64_t)h->C * (o->K + 1) > h->max_rhs)
      return fail(CMTCS_E_INVALID, "C*(K+1) exceeds the handle's max_rhs");
  }
  return CMTCS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// The operator without a handle (cmtcs_apply_noalloc): every buffer beyond the caller's inputs
// and outputs lives in one statically sized device array per GPU.  Host code never uses the
// array's name as an address: the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Dv[t][j] = V[t][j] for j < R, 0 for the padding slots R <= j < Rp.
template <typename VT>
__global__ __launch_bounds__(256) void k_pad_cols(const VT* __restrict__ V, VT* __restrict__ Dv,
                                                  int R, int Rp, int D) {
  const int col = blockIdx.x;
  const int t = col / Rp, j = col % Rp;
  const int d = blockIdx.y * 256 + threadIdx.x;
  if (d >= D) return;
  Dv[(int64_t)col * D + d] = j < R ? V[((int64_t)t * R + j) * D + d] : (VT)0;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

template <typename VT>
cmtcs_status_t apply_noalloc(const cmtcs_problem_t* p, const float* alpha, int R,
                             const int32_t* col_cluster, const void* V, void* AV,
                             hipStream_t st) {
  const int T = p->T, C = p->C, D = p->D;
  const int Rp = col_slots(R);
  int cand[kMaxTileCands];
  op_row_candidates(sizeof(VT) == 8, 0, cand);
  const int fr = cand[0];
  op_row_candidates(sizeof(VT) == 8, 1, cand);
  const int ar = cand[0];
  const int ng = Rp / 16 / group_width(Rp);
  // host tables: W offsets, tiles of both products, cluster of every column slot
  std::vector<int64_t> woff(T + 1, 0);
  std::vector<int4> ft, at;
  for (int t = 0; t < T; ++t) {
    const int np = round16((int)(p->row_off[t + 1] - p->row_off[t]));
    woff[t + 1] = woff[t] + (int64_t)Rp * np;
    for (int n0 = 0; n0 < np; n0 += tile_step(fr))
      for (int cg = 0; cg < ng; ++cg) ft.push_back(make_int4(t, n0, cg, 0));
    for (int d0 = 0; d0 < D; d0 += tile_step(ar))
      for (int cg = 0; cg < ng; ++cg) at.push_back(make_int4(t, d0, cg, 0));
  }
  std::vector<int> colc((size_t)T * Rp, -1);
  for (int t = 0; t < T; ++t)
    for (int j = 0; j < R; ++j) colc[(size_t)t * Rp + j] = col_cluster[(size_t)t * R + j];
  // scratch sections, each 256-byte aligned
  const size_t vec = (size_t)T * Rp * D * sizeof(VT);
  const size_t sz[7] = {sizeof(int64_t) * (T + 1), sizeof(int64_t) * (T + 1),
                        sizeof(int4) * ft.size(), sizeof(int4) * at.size(),
                        sizeof(int) * colc.size(), vec, (size_t)woff[T] * sizeof(VT)};
  size_t off[8] = {0};
  for (int i = 0; i < 7; ++i) off[i + 1] = off[i] + align256(sz[i]);
  const size_t total = off[7] + align256(vec);   // + A V in the padded layout
  if (total > kNoAllocScratchBytes)
    return fail(CMTCS_E_INVALID,
                "problem too large for cmtcs_apply_noalloc: needs " + std::to_string(total) +
                    " bytes of scratch, the limit is " + std::to_string(kNoAllocScratchBytes));
  void* base = nullptr;
  HIP_TRY(scratch_address(&base), "hipGetSymbolAddress(scratch)");
  char* b = (char*)base;
  int64_t* row_off_d = (int64_t*)(b + off[0]);
  int64_t* w_off_d = (int64_t*)(b + off[1]);
  int4* fwd = (int4*)(b + off[2]);
  int4* adj = (int4*)(b + off[3]);
  int* colc_d = (int*)(b + off[4]);
  VT* Dv = (VT*)(b + off[5]);
  VT* W = (VT*)(b + off[6]);
  VT* AD = (VT*)(b + off[7]);
  HIP_TRY(hipMemcpyAsync(row_off_d, p->row_off, sz[0], hipMemcpyHostToDevice, st),
          "hipMemcpyAsync(row_off)");
  HIP_TRY(hipMemcpyAsync(w_off_d, woff.data(), sz[1], hipMemcpyHostToDevice, st),
          "hipMemcpyAsync(w_off)");
  if (!ft.empty())
    HIP_TRY(hipMemcpyAsync(fwd, ft.data(), sz[2], hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(fwd tiles)");
  HIP_TRY(hipMemcpyAsync(adj, at.data(), sz[3], hipMemcpyHostToDevice, st),
          "hipMemcpyAsync(adj tiles)");
  HIP_TRY(hipMemcpyAsync(colc_d, colc.data(), sz[4], hipMemcpyHostToDevice, st),
          "hipMemcpyAsync(colc)");
  // the host tables above are freed on return: wait for their copies
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(noalloc tables)");
  Geometry g;
  g.T = T; g.C = C; g.D = D; g.R = R; g.Rp = Rp;
  g.row_off = row_off_d; g.w_off = w_off_d;
  int64_t np16 = 0;
  for (int t = 0; t < T; ++t) np16 += (p->row_off[t + 1] - p->row_off[t] + 15) / 16;
  g.fwd_split = fwd_split_of(np16, Rp, D);
  hipLaunchKernelGGL((k_pad_cols<VT>), dim3(T * Rp, (D + 255) / 256), dim3(256), 0, st,
                     (const VT*)V, Dv, R, Rp, D);
  HIP_TRY(hipGetLastError(), "launch(pad_cols)");
  const float* phi = (const float*)p->phi;
  HIP_TRY(launch_phi_v<VT>(g, phi, fwd, (int)ft.size(), Dv, W, nullptr, nullptr, fr, st),
          "launch(phi_v)");
  HIP_TRY(launch_phit_w<VT>(g, phi, adj, (int)at.size(), W, Dv, AD, alpha, colc_d, p->beta,
                            nullptr, nullptr, ar, st), "launch(phit_w)");
  CgState s{};
  s.X = AD;
  HIP_TRY(launch_solve_output<VT>(g, s, AV, nullptr, nullptr, 0, nullptr, nullptr, st),
          "launch(copy out)");
  return CMTCS_OK;
}

}  // namespace

extern "C" {

cmtcs_status_t cmtcs_create(cmtcs_handle_t* out, const cmtcs_problem_t* p, void* stream) {
  if (out == nullptr) return fail(CMTCS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (p == nullptr) return fail(CMTCS_E_INVALID, "problem is NULL");
  const int32_t op = enum_bits(p->op), math = enum_bits(p->math);
  const int32_t phi_dtype = enum_bits(p->phi_dtype);
  if (p->T < 1 || p->C < 1) return fail(CMTCS_E_INVALID, "T and C must be >= 1");
  if (p->D < 16 || p->D % 16 != 0 || p->D > 16384)
    return fail(CMTCS_E_INVALID, "D must be a positive multiple of 16, at most 16384");
  if (p->row_off == nullptr) return fail(CMTCS_E_INVALID, "row_off is NULL");
  if (p->row_off[0] != 0) return fail(CMTCS_E_INVALID, "row_off[0] must be 0");
  for (int t = 0; t < p->T; ++t)
    if (p->row_off[t + 1] < p->row_off[t])
      return fail(CMTCS_E_INVALID, "row_off must be non-decreasing");
  const int64_t rows = p->row_off[p->T];
  if (op != CMTCS_OP_DENSE && op != CMTCS_OP_PARTIAL_FOURIER)
    return fail(CMTCS_E_INVALID, "unknown sensing operator");
  const bool fourier = op == CMTCS_OP_PARTIAL_FOURIER;
  if (fourier) {
    if (rows > 0 && (p->freq == nullptr || p->y == nullptr))
      return fail(CMTCS_E_INVALID, "freq and y must be non-NULL");
    if (math != CMTCS_MATH_F64)
      return fail(CMTCS_E_UNSUPPORTED, "partial-Fourier problems run in MATH_F64 only");
    if (p->D < 64 || p->D > 4096 || (p->D & (p->D - 1)) != 0)
      return fail(CMTCS_E_UNSUPPORTED, "partial-Fourier problems need D a power of two, 64..4096");
  } else if (rows > 0 && (p->phi == nullptr || p->y == nullptr)) {
    return fail(CMTCS_E_INVALID, "phi and y must be non-NULL");
  }
  if (!(p->beta > 0.0)) return fail(CMTCS_E_INVALID, "beta must be > 0");
  if (p->max_rhs < 1) return fail(CMTCS_E_INVALID, "max_rhs must be >= 1");
  if (p->max_iters < 1 || p->max_iters > 4096)
    return fail(CMTCS_E_INVALID, "max_iters must be in 1..4096");
  if (p->max_K < 0) return fail(CMTCS_E_INVALID, "max_K must be >= 0");
  if ((int64_t)p->C * (p->max_K + 1) > p->max_rhs && p->max_K > 0)
    return fail(CMTCS_E_INVALID, "max_rhs must be >= C*(max_K+1)");
  if (math != CMTCS_MATH_F64 && math != CMTCS_MATH_F32 && math != CMTCS_MATH_MIXED)
    return fail(CMTCS_E_INVALID, "unknown math mode");
  if (p->phi_resid != nullptr && (math != CMTCS_MATH_MIXED || fourier))
    return fail(CMTCS_E_INVALID, "phi_resid is for MATH_MIXED dense problems only");
  if (math == CMTCS_MATH_MIXED) {
    if (phi_dtype != CMTCS_BF16 && phi_dtype != CMTCS_F16)
      return fail(CMTCS_E_INVALID, "MATH_MIXED needs phi_dtype BF16 or F16");
    if (p->D % 32 != 0) return fail(CMTCS_E_INVALID, "MATH_MIXED needs D a multiple of 32");
  } else if (phi_dtype != CMTCS_F32 && !fourier) {
    return fail(CMTCS_E_INVALID, "MATH_F64 and MATH_F32 take phi_dtype F32");
  }
  for (int t = 0; t < p->T; ++t)
    if (p->row_off[t + 1] - p->row_off[t] > (1 << 30))
      return fail(CMTCS_E_INVALID, "N_t too large");
  if (!fourier) {
    // the operator products address each task's blocks with 32-bit byte offsets
    const int64_t lim = int64_t(1) << 32, slots = col_slots(p->max_rhs);
    if (slots * p->D * 8 >= lim)
      return fail(CMTCS_E_UNSUPPORTED, "column slots * D * 8 bytes must be below 4 GiB");
    for (int t = 0; t < p->T; ++t) {
      const int64_t nt = p->row_off[t + 1] - p->row_off[t];
      if ((nt + 15) / 16 * 16 * p->D * 4 >= lim)
        return fail(CMTCS_E_UNSUPPORTED, "a task's Phi block (N_t * D * 4 bytes) must be below 4 GiB");
      if (slots * ((nt + 15) / 16 * 16) * 8 >= lim)
        return fail(CMTCS_E_UNSUPPORTED, "a task's W block (slots * N_t * 8 bytes) must be below 4 GiB");
    }
  }

  cmtcs_handle_s* h = new (std::nothrow) cmtcs_handle_s();
  if (h == nullptr) return fail(CMTCS_E_NOMEM, "host allocation failed");
  h->T = p->T; h->C = p->C; h->D = p->D; h->beta = p->beta; h->math = (cmtcs_math_t)math;
  h->max_rhs = p->max_rhs; h->max_iters = p->max_iters; h->max_K = p->max_K;
  h->Rp_max = col_slots(p->max_rhs);
  h->vbytes = math == CMTCS_MATH_F64 ? 8 : 4;
  h->row_off.assign(p->row_off, p->row_off + p->T + 1);
  for (int t = 0; t < p->T; ++t) h->np16 += (h->row_off[t + 1] - h->row_off[t] + 15) / 16;
  h->phi_dtype = (cmtcs_dtype_t)phi_dtype;
  h->phi = (const float*)p->phi;
  h->phi_res = p->phi_resid != nullptr ? p->phi_resid : (const float*)p->phi;
  h->y = p->y;
  h->fourier = fourier;
  h->freq = p->freq;
  h->st = (hipStream_t)stream;

  const size_t T = h->T, C = h->C, D = h->D, Rpm = h->Rp_max, it = h->max_iters;
  size_t np_sum = 0, fwd_max = 0;
  const bool f64 = h->math == CMTCS_MATH_F64;
  const size_t ngm = (size_t)h->ngroups(h->Rp_max);
  // tile tables are sized for the smallest tile of either product
  int min_rows = 1 << 30;
  int cand[2][kMaxTileCands], ncand[2];
  for (int kind = 0; kind < 2; ++kind) {
    ncand[kind] = op_row_candidates(f64, kind, cand[kind]);
    for (int i = 0; i < ncand[kind]; ++i) min_rows = std::min(min_rows, tile_step(cand[kind][i]));
  }
  h->fwd_rows = cand[0][0];
  h->adj_rows = cand[1][0];
  // CMTCS_SLQ_LDS_BYTES lowers the SLQ kernel's LDS budget (0: every tridiagonal in the HBM
  // workspace, the form that runs past 4096 CG steps); read here, where the workspace is sized
  if (const char* sl = std::getenv("CMTCS_SLQ_LDS_BYTES"))
    h->slq_lds = std::max(0L, std::min(kSlqLdsBytes, std::atol(sl)));
  const char* at = std::getenv("CMTCS_AUTOTUNE");
  h->autotune = !(at != nullptr && at[0] == '0');
  // CMTCS_COMPACT=0 makes the CG loop's products multiply every column slot (for comparison:
  // the results are the same bit for bit)
  const char* cp = std::getenv("CMTCS_COMPACT");
  h->compact = !(cp != nullptr && cp[0] == '0');
  // CMTCS_TILES="fwd,adj" pins both tile heights (each one of the supported candidates) and
  // turns the autotuner off; unsupported values leave the defaults in place
  if (const char* pin = std::getenv("CMTCS_TILES")) {
    int f = 0, a = 0;
    if (std::sscanf(pin, "%d,%d", &f, &a) == 2) {
      bool okf = false, oka = false;
      for (int i = 0; i < ncand[0]; ++i) okf = okf || cand[0][i] == f;
      for (int i = 0; i < ncand[1]; ++i) oka = oka || cand[1][i] == a;
      if (okf && oka) { h->fwd_rows = f; h->adj_rows = a; h->autotune = false; }
    }
  }
  for (size_t t = 0; t < T; ++t) {
    const size_t np = (size_t)round16((int)(h->row_off[t + 1] - h->row_off[t]));
    np_sum += np;
    fwd_max += (np + min_rows - 1) / min_rows * ngm;
  }
  const size_t adj_max = T * ((D + min_rows - 1) / min_rows) * ngm;
  const size_t vec = T * Rpm * D * h->vbytes;
  const size_t P = T * C * (size_t)h->max_K;
  hipError_t e = hipSuccess;
  auto A = [&](auto** ptr, size_t bytes) {
    if (e == hipSuccess) e = h->alloc(ptr, bytes);
  };
  A(&h->row_off_d, sizeof(int64_t) * (T + 1));
  A(&h->w_off_d, sizeof(int64_t) * (T + 1));
  A(&h->X, vec);
  if (fourier) {
    // the CG state lives in the solve kernel; the multiplier counts per task
    A(&h->hcount, sizeof(int) * T * D);
    A(&h->bad_freq, sizeof(int));
  } else {
    A(&h->Rv, vec); A(&h->Dv, vec); A(&h->AD, vec);
    A(&h->W, Rpm * np_sum * h->vbytes);
    if (f64) {
      h->pt_off.assign(T + 1, 0);
      for (size_t t = 0; t < T; ++t) {
        const int np = round16((int)(h->row_off[t + 1] - h->row_off[t]));
        h->pt_off[t + 1] = h->pt_off[t] + np;
        h->max_np = std::max(h->max_np, np);
      }
      A(&h->phiT, sizeof(float) * D * np_sum);
      A(&h->pt_off_d, sizeof(int64_t) * (T + 1));
    }
    A(&h->mbase, sizeof(double) * T * D);
    A(&h->mdiag, sizeof(double) * T * C * D);
    A(&h->slogm, sizeof(double) * T * C);
  }
  A(&h->b, T * D * h->vbytes);
  A(&h->rr, sizeof(double) * T * Rpm);
  A(&h->thr, sizeof(double) * T * Rpm);
  A(&h->state, T * Rpm);
  A(&h->iters, sizeof(int) * T * Rpm);
  A(&h->gam, sizeof(double) * it * T * Rpm);
  A(&h->xi, sizeof(double) * it * T * Rpm);
  A(&h->act, sizeof(int) * (it + 1) * T);
  A(&h->colc, sizeof(int) * T * (Rpm + (size_t)h->max_rhs));   // [T][Rp] + map staging
  if (!fourier) {
    A(&h->fwd_tiles, sizeof(int4) * fwd_max);
    A(&h->adj_tiles, sizeof(int4) * adj_max);
  }
  // SLQ tridiagonals of runs too long for LDS
  A(&h->slq_ws, std::max<size_t>(16, slq_workspace_bytes((long)P, (int)it, h->slq_lds)));
  A(&h->key_d, sizeof(uint64_t));
  A(&h->tau, sizeof(double) * P);
  A(&h->rmin, sizeof(double) * P);
  A(&h->rmax, sizeof(double) * P);
  A(&h->ok, P);
  A(&h->keff, sizeof(int) * T * C);
  A(&h->slog, sizeof(double) * C);
  A(&h->lconst, sizeof(double) * std::max<size_t>(1, T));
  if (h->math == CMTCS_MATH_MIXED) {
    size_t np32_sum = 0, f16_max = 0;
    for (size_t t = 0; t < T; ++t) {
      const size_t np = (size_t)((h->row_off[t + 1] - h->row_off[t] + 31) / 32 * 32);
      np32_sum += (size_t)ld16((int64_t)np);
      h->max_np32 = std::max(h->max_np32, (int)np);
      f16_max += (np + kRows16 - 1) / kRows16 * ngm;
    }
    A(&h->phi16, 2 * (size_t)ld16(D) * (size_t)rows);
    A(&h->phiT16, 2 * D * np32_sum);
    A(&h->D16, 2 * T * Rpm * (size_t)ld16(D));
    A(&h->W16, 2 * Rpm * np32_sum);
    A(&h->w16_off_d, sizeof(int64_t) * (T + 1));
    A(&h->fwd16_tiles, sizeof(int4) * f16_max);
    A(&h->adj16_tiles, sizeof(int4) * T * ((D + kRows16 - 1) / kRows16) * ngm);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->act_host, sizeof(int) * T);
  if (e != hipSuccess) {
    delete h;
    if (e == hipErrorOutOfMemory) return fail(CMTCS_E_NOMEM, "workspace allocation failed");
    return hip_fail(e, "hipMalloc(workspace)");
  }
  e = hipMemcpyAsync(h->row_off_d, h->row_off.data(), sizeof(int64_t) * (T + 1),
                     hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess && h->pt_off_d != nullptr)   // from the handle's own vector
    e = hipMemcpyAsync(h->pt_off_d, h->pt_off.data(), sizeof(int64_t) * (T + 1),
                       hipMemcpyHostToDevice, h->st);
  int bad = 0;
  if (e == hipSuccess) {
    const Geometry g = h->geom(1, 16);
    if (fourier)
      e = launch_fourier_setup(g, h->freq, h->y, h->beta, (double*)h->b, h->hcount, h->bad_freq,
                               h->st);
    else if (f64) e = launch_rhs<double>(g, h->phi, h->y, h->beta, (double*)h->b, h->st);
    else e = launch_rhs<float>(g, h->phi, h->y, h->beta, (float*)h->b, h->st);
    if (e == hipSuccess && !fourier) e = launch_colnorm(g, h->phi, h->beta, h->mbase, h->st);
    if (e == hipSuccess)
      e = launch_log_norm_const(T, h->y, h->row_off_d, fourier ? 2 : 1, h->beta, h->lconst,
                                h->st);
  }
  if (e == hipSuccess && fourier)
    e = hipMemcpyAsync(&bad, h->bad_freq, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "cmtcs_create");
  }
  if (bad != 0) {
    delete h;
    return fail(CMTCS_E_INVALID, "freq entries must be in 0..D-1");
  }
  if (h->math == CMTCS_MATH_MIXED) {
    // 16-bit tables and offsets, then the transposed 16-bit copy of Phi
    cmtcs_status_t rs = h->prepare(h->Rp_max);
    if (rs != CMTCS_OK) {
      delete h;
      return rs;
    }
    const Geometry g16 = h->geom16(1, h->Rp_max);
    const int64_t lp = ld16(h->D);
    if (h->phi_dtype == CMTCS_BF16) {
      e = launch_round16<__bf16>((const float*)h->phi, h->D, h->phi16, lp, rows, h->D, h->st);
      if (e == hipSuccess)
        e = launch_transpose16<__bf16>(g16, h->phi16, h->phiT16, h->max_np32, h->st);
    } else {
      e = launch_round16<_Float16>((const float*)h->phi, h->D, h->phi16, lp, rows, h->D, h->st);
      if (e == hipSuccess)
        e = launch_transpose16<_Float16>(g16, h->phi16, h->phiT16, h->max_np32, h->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(e, "cmtcs_create (transpose)");
    }
  }
  *out = h;
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_destroy(cmtcs_handle_t h) {
  if (h == nullptr) return CMTCS_OK;
  hipError_t e = hipStreamSynchronize(h->st);
  delete h;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(destroy)");
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_estep(cmtcs_handle_t h, const float* alpha, const double* log_pi,
                           const cmtcs_opts_t* opts, float* mu, float* s, double* logdet,
                           double* ell, double* q, cmtcs_cg_stats_t* stats) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  cmtcs_status_t rs = check_opts(h, opts, true);
  if (rs != CMTCS_OK) return rs;
  if (!alpha || !log_pi || !mu || !s || !logdet || !ell || !q)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  if (h->math == CMTCS_MATH_F64)
    return h->estep<double>(alpha, log_pi, *opts, mu, s, logdet, ell, q, stats);
  return h->estep<float>(alpha, log_pi, *opts, mu, s, logdet, ell, q, stats);
}

cmtcs_status_t cmtcs_mstep(cmtcs_handle_t h, const float* mu, const float* s, const double* q,
                           const cmtcs_opts_t* opts, float* alpha_inout) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (opts == nullptr) return fail(CMTCS_E_INVALID, "opts is NULL");
  if (!(opts->alpha_max > 0.0)) return fail(CMTCS_E_INVALID, "alpha_max must be > 0");
  if (!mu || !s || !q || !alpha_inout)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  HIP_TRY(launch_mstep(h->T, h->C, h->D, mu, s, q, opts->alpha_max, alpha_inout, h->st),
          "launch(mstep)");
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_mstep_pi(cmtcs_handle_t h, const double* q, double* log_pi) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (!q || !log_pi) return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  HIP_TRY(launch_update_pi(h->T, h->C, q, log_pi, h->st), "launch(mstep_pi)");
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_log_likelihood(cmtcs_handle_t h, const double* ell, const double* log_pi,
                                    double* L_task, double* L_mean) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (!ell || !log_pi) return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  if (!L_task && !L_mean) return CMTCS_OK;
  HIP_TRY(launch_log_likelihood(h->T, h->C, ell, log_pi, h->lconst, L_task, L_mean, h->st),
          "launch(log_likelihood)");
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_em_iter(cmtcs_handle_t h, float* alpha_inout, const double* log_pi,
                             const cmtcs_opts_t* opts, float* mu, float* s, double* logdet,
                             double* ell, double* q) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  cmtcs_status_t rs = check_opts(h, opts, true);
  if (rs != CMTCS_OK) return rs;
  if (!(opts->alpha_max > 0.0)) return fail(CMTCS_E_INVALID, "alpha_max must be > 0");
  if (!alpha_inout || !log_pi || !mu || !s || !logdet || !ell || !q)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  if (h->math == CMTCS_MATH_F64)
    return h->em_iter<double>(alpha_inout, log_pi, *opts, mu, s, logdet, ell, q);
  return h->em_iter<float>(alpha_inout, log_pi, *opts, mu, s, logdet, ell, q);
}

cmtcs_status_t cmtcs_solve(cmtcs_handle_t h, const float* alpha, int32_t R_per_task,
                           const int32_t* col_cluster, const void* B, void* X, double* gamma,
                           double* xi, const cmtcs_opts_t* opts, cmtcs_cg_stats_t* stats) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  cmtcs_status_t rs = check_opts(h, opts, false);
  if (rs != CMTCS_OK) return rs;
  if (R_per_task < 1 || R_per_task > h->max_rhs)
    return fail(CMTCS_E_INVALID, "R_per_task must be in 1..max_rhs");
  if (!alpha || !col_cluster || !B || !X)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  for (int64_t i = 0; i < (int64_t)h->T * R_per_task; ++i)
    if (col_cluster[i] < 0 || col_cluster[i] >= h->C)
      return fail(CMTCS_E_INVALID, "col_cluster entries must be in 0..C-1");
  if (h->math == CMTCS_MATH_F64)
    return h->solve<double>(alpha, R_per_task, col_cluster, B, X, gamma, xi, *opts, stats);
  return h->solve<float>(alpha, R_per_task, col_cluster, B, X, gamma, xi, *opts, stats);
}

cmtcs_status_t cmtcs_rhs(cmtcs_handle_t h, void* b) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (b == nullptr) return fail(CMTCS_E_INVALID, "b is NULL");
  HIP_TRY(hipMemcpyAsync(b, h->b, h->vbytes * h->T * h->D, hipMemcpyDeviceToDevice, h->st),
          "hipMemcpyAsync(rhs)");
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_grad(cmtcs_handle_t h, int32_t R_per_task, const int32_t* col_cluster,
                          const void* X, const void* Lam, double y_coef, float* dalpha,
                          float* dphi) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (R_per_task < 1 || 2 * (int64_t)R_per_task > h->max_rhs)
    return fail(CMTCS_E_INVALID, "R_per_task must be in 1..max_rhs/2");
  if (!col_cluster || !X || !Lam) return fail(CMTCS_E_INVALID, "a required argument is NULL");
  if (h->fourier)
    return fail(CMTCS_E_UNSUPPORTED, "cmtcs_grad is not available for partial-Fourier problems");
  for (int64_t i = 0; i < (int64_t)h->T * R_per_task; ++i)
    if (col_cluster[i] < 0 || col_cluster[i] >= h->C)
      return fail(CMTCS_E_INVALID, "col_cluster entries must be in 0..C-1");
  if (h->math == CMTCS_MATH_F64)
    return h->grad<double>(R_per_task, col_cluster, X, Lam, y_coef, dalpha, dphi);
  return h->grad<float>(R_per_task, col_cluster, X, Lam, y_coef, dalpha, dphi);
}

cmtcs_status_t cmtcs_apply(cmtcs_handle_t h, const float* alpha, int32_t R_per_task,
                           const int32_t* col_cluster, const void* V, void* AV) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (R_per_task < 1 || R_per_task > h->max_rhs)
    return fail(CMTCS_E_INVALID, "R_per_task must be in 1..max_rhs");
  if (!alpha || !col_cluster || !V || !AV)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  for (int64_t i = 0; i < (int64_t)h->T * R_per_task; ++i)
    if (col_cluster[i] < 0 || col_cluster[i] >= h->C)
      return fail(CMTCS_E_INVALID, "col_cluster entries must be in 0..C-1");
  if (h->math == CMTCS_MATH_F64) return h->apply<double>(alpha, R_per_task, col_cluster, V, AV);
  return h->apply<float>(alpha, R_per_task, col_cluster, V, AV);
}

cmtcs_status_t cmtcs_profile(cmtcs_handle_t h, int32_t enable, double* totals_ms,
                             int64_t* counts) {
  if (h == nullptr) return fail(CMTCS_E_INVALID, "handle is NULL");
  if (enable == 1) {
    if (!h->ev_made) {
      for (auto& row : h->ev)
        for (auto& e : row) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
      h->ev_made = true;
    }
    HIP_TRY(h->harvest(), "profile events");
    for (int k = 0; k < 3; ++k) { h->prof_ms[k] = 0; h->prof_n[k] = 0; }
    h->prof_on = true;
  } else if (enable == 0) {
    HIP_TRY(h->harvest(), "profile events");
    h->prof_on = false;
  }
  if (totals_ms != nullptr || counts != nullptr) {
    HIP_TRY(hipStreamSynchronize(h->st), "hipStreamSynchronize(profile)");
    HIP_TRY(h->harvest(), "profile events");
    for (int k = 0; k < 3; ++k) {
      if (totals_ms) totals_ms[k] = h->prof_ms[k];
      if (counts) counts[k] = h->prof_n[k];
    }
  }
  return CMTCS_OK;
}

cmtcs_status_t cmtcs_apply_noalloc(const cmtcs_problem_t* p, const float* alpha,
                                   int32_t R_per_task, const int32_t* col_cluster, const void* V,
                                   void* AV, void* stream) {
  if (p == nullptr) return fail(CMTCS_E_INVALID, "problem is NULL");
  const int32_t op = enum_bits(p->op), math = enum_bits(p->math);
  if (p->T < 1 || p->C < 1) return fail(CMTCS_E_INVALID, "T and C must be >= 1");
  if (p->D < 16 || p->D % 16 != 0 || p->D > 16384)
    return fail(CMTCS_E_INVALID, "D must be a positive multiple of 16, at most 16384");
  if (op != CMTCS_OP_DENSE)
    return fail(CMTCS_E_UNSUPPORTED, "cmtcs_apply_noalloc takes dense problems only");
  if (math != CMTCS_MATH_F64 && math != CMTCS_MATH_F32)
    return fail(CMTCS_E_UNSUPPORTED, "cmtcs_apply_noalloc runs MATH_F64 or MATH_F32");
  if (enum_bits(p->phi_dtype) != CMTCS_F32)
    return fail(CMTCS_E_INVALID, "phi_dtype must be F32");
  if (!(p->beta > 0.0)) return fail(CMTCS_E_INVALID, "beta must be > 0");
  if (p->row_off == nullptr || p->row_off[0] != 0)
    return fail(CMTCS_E_INVALID, "row_off must be non-NULL with row_off[0] = 0");
  for (int t = 0; t < p->T; ++t)
    if (p->row_off[t + 1] < p->row_off[t])
      return fail(CMTCS_E_INVALID, "row_off must be non-decreasing");
  if (p->row_off[p->T] > 0 && p->phi == nullptr) return fail(CMTCS_E_INVALID, "phi is NULL");
  if (R_per_task < 1) return fail(CMTCS_E_INVALID, "R_per_task must be >= 1");
  if (!alpha || !col_cluster || !V || !AV)
    return fail(CMTCS_E_INVALID, "a required array argument is NULL");
  for (int64_t i = 0; i < (int64_t)p->T * R_per_task; ++i)
    if (col_cluster[i] < 0 || col_cluster[i] >= p->C)
      return fail(CMTCS_E_INVALID, "col_cluster entries must be in 0..C-1");
  {
    // 32-bit per-task offsets of the operator products (as checked by cmtcs_create)
    const int64_t lim = int64_t(1) << 32, slots = col_slots(R_per_task);
    if (slots * p->D * 8 >= lim)
      return fail(CMTCS_E_UNSUPPORTED, "column slots * D * 8 bytes must be below 4 GiB");
    for (int t = 0; t < p->T; ++t) {
      const int64_t nt = p->row_off[t + 1] - p->row_off[t];
      if ((nt + 15) / 16 * 16 * p->D * 4 >= lim || slots * ((nt + 15) / 16 * 16) * 8 >= lim)
        return fail(CMTCS_E_UNSUPPORTED, "a task's block must be below 4 GiB");
    }
  }
  hipStream_t st = (hipStream_t)stream;
  if (enum_bits(p->math) == CMTCS_MATH_F64)
    return apply_noalloc<double>(p, alpha, R_per_task, col_cluster, V, AV, st);
  return apply_noalloc<float>(p, alpha, R_per_task, col_cluster, V, AV, st);
}

cmtcs_status_t cmtcs_tiles(cmtcs_handle_t h, int32_t* rows) {
  if (h == nullptr || rows == nullptr) return fail(CMTCS_E_INVALID, "NULL argument");
  rows[0] = h->fwd_rows;
  rows[1] = h->adj_rows;
  return CMTCS_OK;
}

const char* cmtcs_last_error(void) { return g_err.c_str(); }

const char* cmtcs_version(void) { return "cmtcs 0.1.0 (gfx950)"; }

}  // extern "C"
