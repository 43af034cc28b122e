// Host driver and C ABI of libfab (see include/fab.h for the contract).
//
// One fab_solve runs the restarted loop of Algorithm 2.  Every cycle is the same sequence of
// kernel launches (cycle start, m steps of sketch + orthogonalisation + update, cycle-end small
// work, fused pass, convergence test), so a cycle is captured once as a hipGraph and replayed;
// the host reads one small report per cycle to decide whether to stop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fab.h"
#include "fab_internal.h"

namespace fab {
hipError_t launch_spmv_sketch(hipStream_t, int dtype, int mode, int grid, int n, const int* rp, const int* ci,
                              const int16_t* cr, const void* va, const void* x, void* y, int d, int zeta, uint64_t seed,
                              double* parts, const State* st, int nb, int G, size_t bs, int nts = 0,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_reduce_parts(hipStream_t, int e0, int len, int nparts, const double* parts, double* out,
                               const State* st, int skip, int nb, size_t bs);
size_t spmv_sketch_lds(int dtype, int mode, int d, int G, int zeta, bool c16);
int spmv_blocks_per_cu(int dtype, int mode, int d, int G, int zeta, bool c16);
hipError_t configure_cycle_kernels();
hipError_t configure_step_kernels();
size_t group_lds_max();
hipError_t launch_orth(hipStream_t, int j, int k, int m, int d, const double* uraw, double* U, double* R,
                       State* st, int nb, size_t bs);
hipError_t launch_update(hipStream_t, int dtype, int grid, int n, int j, int k, void* W, const State* st, int nb,
                         size_t bs, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_orth_update(hipStream_t, int dtype, int num_cu, int n, int j, int k, int m, int d, void* W,
                              const double* uraw, double* U, double* R, double* G, State* st, int nb, size_t bs,
                              const double* parts, int nparts, int nts, hipEvent_t e0 = nullptr,
                              hipEvent_t e1 = nullptr);
hipError_t launch_gram(hipStream_t, int dtype, int grid, int n, int j1, const void* V, const void* z,
                       double* slots, int want_norm, const State* st);
hipError_t launch_cgs_update(hipStream_t, int dtype, int grid, int n, int j, int m, void* V, const double* slots,
                             double* slots_zero, double* norm_slots, int want_norm, double* R, State* st);
hipError_t launch_plain_finish(hipStream_t, int j, int m, double* norm_slots, double* R, State* st);
hipError_t launch_scale_col(hipStream_t, int dtype, int grid, int n, void* v, const double* s_ptr,
                            const State* st, int nb, size_t bs);
hipError_t launch_zero(hipStream_t, double* p, size_t count);
hipError_t launch_zero_strided(hipStream_t, double* p, size_t count, int reps, size_t step_bytes);
hipError_t launch_rule(hipStream_t, int fun, int nt, const double* tvals, int n_main, double lo, double hi,
                       cplx* rz, cplx* rw, cplx* psi, State* st, int nb, size_t bs);
hipError_t launch_copy_in(hipStream_t, int dtype, int grid, int n, const void* b, int64_t ldb, void* w0, int nb,
                          size_t bs);
hipError_t launch_sqnorm(hipStream_t, int dtype, int grid, int n, const void* v, double* slots);
hipError_t launch_start(hipStream_t, int d, int m, int plain, const double* sv, double* slots_start,
                        double* slots_step, size_t step_len, double* U, double* R, State* st, int nb, size_t bs);

hipError_t launch_small(hipStream_t, const SmallArgs& a, int nb, const GrowBuffers* grow);
hipError_t launch_pass(hipStream_t, int dtype, int grid, int n, int m, int nt, int dn, const double* C, void* W,
                       double* x, int64_t ldx, double* parts, const State* st, int nb, size_t bs, const PassSketch& ps);
hipError_t launch_final(hipStream_t, int nt, int dn, double tol, double div_limit, double uround, const double* red,
                        State* st, Report* rep, int nb, size_t bs);
hipError_t launch_sketch_table(hipStream_t, int64_t col0, int64_t count, int d, int zeta, uint64_t seed, int* rows,
                               int8_t* signs);
hipError_t launch_dot(hipStream_t, int64_t n, const double* x, const double* y, double* part, int max_blocks,
                      double* out);
hipError_t launch_csr_validate(hipStream_t, int n, int nnz, const int* rowptr, const int* colind, int* flag);
hipError_t launch_col_offsets(hipStream_t, int n, const int* rowptr, const int* colind, int16_t* off, int* flag);
size_t transpose_scan_blocks(int64_t len);
hipError_t launch_transpose(hipStream_t, int dtype, int n, int nnz, const int* rowptr, const int* colind,
                            const void* vals, int* rowptrT, int* colT, void* valT, int* cursor, int* sums);
}  // namespace fab

constexpr int kDotBlocks = 1024;  // partial sums of fab_dot (fixed grid: reproducible bits)

using namespace fab;

// Timing events: [2j, 2j+1] around step j's product + sketch, [kTevUpdate + 2j, +1] around its window
// update (the fused Gram-Schmidt + update, or the update alone), kTevEnd at the end of the step loop.
constexpr int kTevUpdate = 2 * kMaxM, kTevEnd = 4 * kMaxM;

struct GraphKey {
  uint64_t op;  // fab_op::serial
  const void* work;
  const void* x;
  int64_t n;
  int m, k, d, zeta, nt, fun, method, nq, dtype;
  uint64_t seed;
  double tol;
  int timing, nb, G, nts;
  int64_t ldx;
  size_t bs;
  double div_limit;
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

struct fab_ctx {
  int device = 0;
  double* scratch = nullptr;  // this device's copy of `scratch` (fab_sketch_apply_noalloc)
  hipStream_t user = nullptr;
  hipStream_t work = nullptr;
  hipEvent_t ev = nullptr;
  Report* h_rep = nullptr;
  double* d_part = nullptr;  // kDotBlocks partial sums of fab_dot (device)
  double* h_t = nullptr;  // pinned staging for the time points
  int num_cu = 256;
  // benchmark timing: events around each SpMV+sketch launch and each window-update launch (2 each
  // per step; see kTevUpdate) and at the loop end (kTevEnd)
  bool timing = false;
  bool timing_loop_only = false;  // fab_timing_enable(ctx, 2): events at the step loops' ends only
  std::vector<hipEvent_t> tev;
  double t_spmv_ms = 0.0, t_loop_ms = 0.0, t_upd_ms = 0.0;
  int64_t t_spmv_n = 0, t_loop_n = 0, t_upd_n = 0;
  struct Cached {
    GraphKey key;
    hipGraphExec_t exec;
  };
  struct Tuned {  // autotuned members per block of the fused kernel, per operator and batch shape
    uint64_t op;  // fab_op::serial (a destroyed operator's address can be reused by a new one)
    int64_t n;
    int nb, d, zeta, dtype, G;
  };
  std::vector<Tuned> tuned;
  int force_group = 0;  // fab_batch_group: 0 = autotune
  double div_limit = kDivergedEst;  // fab_divergence_limit: relative increment that abandons a solve
  // ragged solves: branch streams, the fork/join events around the branch graphs, and their cache
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  std::vector<uintptr_t> ragged_key;
  std::vector<hipGraphExec_t> ragged_execs;  // one per branch stream
  std::vector<Cached> graphs;
};

struct fab_op {
  fab_ctx* ctx;
  int64_t n, nnz;
  const int32_t* rowptr;
  const int32_t* colind;
  const void* vals;
  int dtype;
  void* owned;  // device storage the library allocated for this operator (transposes), else null
  uint64_t serial = 0;  // unique per operator for the process: keys the cached graphs, whose kernel
                        // arguments hold this operator's arrays (an address can be reused after a destroy)
  int16_t* colrel = nullptr;  // library-owned 16-bit column offsets (see derive_col_offsets), else null
  int nts = 0;  // the step's z and basis stores non-temporal (fab_op_store_policy; set by size_policy)
};

// The memory-side cache (MALL) of the device: 256 MB on MI355X.
constexpr int64_t kMallBytes = (int64_t)256 << 20;

// Cache policy of a single solve's step by operator size: CSR arrays as the products read them
// (values, the 16-bit offsets when present else the int32 columns, row pointers) larger than the
// memory-side cache stream through it on every product, and the step's vectors then store
// non-temporal.  Measured: default policy 3% faster on a 154 MB CSR, non-temporal 2-3% per cycle
// faster on a 1.4 GB one.
static int size_policy(const fab_op* A) {
  const int64_t es = A->dtype == FAB_F64 ? 8 : 4, ib = A->colrel ? 2 : 4;
  return A->nnz * (es + ib) + 4 * (A->n + 1) > kMallBytes ? 1 : 0;
}

static uint64_t next_op_serial() {
  static std::atomic<uint64_t> counter{0};
  return ++counter;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

static int rule_nodes(int fun, const fab_params* p) {
  return (p->n_quad > 0) ? p->n_quad : (fun == FAB_COS_SQRT ? kRuleCosSqrt : kRuleMain);
}

// Functions of a time parameter t (h_t): exp(-t z), phi_1(-t z), cos(t sqrt z); z^(-1/2) has none.
static bool timed_fun(int fun) { return fun == FAB_EXP_NEG || fun == FAB_PHI1_NEG || fun == FAB_COS_SQRT; }

static Layout make_layout(int64_t n, int dtype, const fab_params* p, int fun, int nt) {
  Layout L{};
  const size_t es = dtype == 0 ? 8 : 4;
  const int m = p->m;
  const int d = (p->method == FAB_PLAIN_RESTART) ? 1 : p->d;
  const int N = rule_nodes(fun, p);
  L.nq = rule_is_half(fun) ? N / 2 : N;
  L.nsys = nt * L.nq;
  const bool plain = p->method == FAB_PLAIN_RESTART;
  const size_t step_len = (size_t)kSlots * std::max(d, kMaxM + 2);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.W = take(wcol(n, (int)es) * (m + 1) * es);
  L.U = take((size_t)d * (m + 1) * 8);
  L.R = take((size_t)(m + 1) * m * 8);
  // zeroed at set-up from slots_step up to T: the plain comparator's atomic accumulators, the
  // reduced sketches and norms, the state
  L.slots_step = take(plain ? 2 * step_len * 8 : 0);
  L.slots_start = take(plain ? (size_t)kSlots * 8 : 0);
  L.uraw = take((size_t)d * 8);
  L.red = take((size_t)(d + 2 * kMaxNt) * 8);
  L.state = take(sizeof(State));
  L.T = take((size_t)(m + 1) * (m + 1) * 8);
  L.Ut = take((size_t)d * (m + 1) * 8);
  L.X = take((size_t)m * m * 8);
  L.C = take((size_t)(m + 1) * (nt + 1) * 8);
  L.rule_z = take((size_t)L.nsys * sizeof(cplx));
  L.rule_w = take((size_t)L.nsys * sizeof(cplx));
  L.psi = take((size_t)L.nsys * sizeof(cplx));
  L.gbuf = take((size_t)L.nsys * m * 8 + (size_t)nt * 8 /* t values */);
  // growing restart: blocks (kGrowRows x m), couplings and sizes per cycle
  L.grow = take(p->method == FAB_SKETCHED_GROWING ? (size_t)kGrowRows * m * 8 + (size_t)kGrowRows * 12 : 0);
  L.G = take((size_t)(m + 1) * (m + 1) * 8);
  // per-block partials (k_reduce_parts): the sketch entries [0, d), then the pass's norms
  L.parts = take((size_t)kMaxParts * (d + 2 * kMaxNt) * 8);
  L.total = off;
  return L;
}

static fab_status check_params(const fab_op* A, const fab_params* p, int fun, int nt) {
  if (!A || !p) return FAB_E_INVALID;
  if (p->m < 1 || p->m > kMaxM) return FAB_E_INVALID;
  if (p->method != FAB_SKETCHED && p->method != FAB_PLAIN_RESTART && p->method != FAB_SKETCHED_GROWING)
    return FAB_E_INVALID;
  if (p->method != FAB_PLAIN_RESTART) {
    if (p->k < 1 || p->k > p->m) return FAB_E_INVALID;
    if (p->d < p->m + 1 || p->d > kMaxD) return FAB_E_INVALID;
    if (p->zeta < 1 || p->zeta > 32 || p->zeta > p->d) return FAB_E_INVALID;
  }
  if (!(p->tol >= 0.0) || p->max_cycles < 1) return FAB_E_INVALID;
  if (p->n_quad != 0 && (p->n_quad < 8 || p->n_quad > 512 || (p->n_quad % 8) != 0)) return FAB_E_INVALID;
  if (fun == FAB_EXP_NEG || fun == FAB_PHI1_NEG) {
    if (nt < 1 || nt > kMaxNt) return FAB_E_INVALID;
  } else if (fun == FAB_COS_SQRT) {  // the ellipse rule needs the spectral interval
    if (nt < 1 || nt > kMaxNt) return FAB_E_INVALID;
    if (!(p->spec_lo >= 0.0) || !(p->spec_hi > p->spec_lo) || !std::isfinite(p->spec_hi)) return FAB_E_INVALID;
  } else if (fun == FAB_INVSQRT) {
    if (nt != 1) return FAB_E_INVALID;
    if (!(p->spec_lo > 0.0) || !(p->spec_hi >= p->spec_lo) || !std::isfinite(p->spec_hi)) return FAB_E_INVALID;
  } else {
    return FAB_E_INVALID;
  }
  if (A->n >= (int64_t)1 << 31) return FAB_E_UNSUPPORTED;
  if (p->method == FAB_SKETCHED_GROWING &&
      (fun != FAB_EXP_NEG || (int64_t)p->max_cycles * p->m > kGrowRows))
    return FAB_E_UNSUPPORTED;
  return FAB_OK;
}

static int stream_grid(int64_t n, int cap) {
  int64_t g = (n + kThreads - 1) / kThreads;
  g = std::min<int64_t>(g, cap);
  g = ((g + kXcds - 1) / kXcds) * kXcds;
  return (int)std::max<int64_t>(g, kXcds);
}

struct Ptrs {
  char* base;
  void* W;
  double *U, *R, *slots_step, *slots_start, *uraw, *red, *parts, *T, *Ut, *X, *C, *gbuf, *tvals, *G;
  State* st;
  cplx *rz, *rw, *psi;
  size_t step_len;
};

static Ptrs carve(void* work, const Layout& L, const fab_params* p, int nt) {
  Ptrs q{};
  q.base = (char*)work;
  q.W = q.base + L.W;
  q.U = (double*)(q.base + L.U);
  q.R = (double*)(q.base + L.R);
  q.slots_step = (double*)(q.base + L.slots_step);
  q.slots_start = (double*)(q.base + L.slots_start);
  q.uraw = (double*)(q.base + L.uraw);
  q.red = (double*)(q.base + L.red);
  q.parts = (double*)(q.base + L.parts);
  q.st = (State*)(q.base + L.state);
  q.T = (double*)(q.base + L.T);
  q.Ut = (double*)(q.base + L.Ut);
  q.X = (double*)(q.base + L.X);
  q.C = (double*)(q.base + L.C);
  q.rz = (cplx*)(q.base + L.rule_z);
  q.rw = (cplx*)(q.base + L.rule_w);
  q.psi = (cplx*)(q.base + L.psi);
  q.gbuf = (double*)(q.base + L.gbuf);
  q.tvals = q.gbuf + (size_t)L.nsys * p->m;
  q.G = (double*)(q.base + L.G);
  const int d = (p->method == FAB_PLAIN_RESTART) ? 1 : p->d;
  q.step_len = (size_t)kSlots * std::max(d, kMaxM + 2);
  return q;
}

// Text of the last failing HIP call on this host thread (fab_last_error).
static thread_local char g_last_error[256] = "";

static fab_status hip_fail(hipError_t e, const char* expr, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d) at api.hip:%d: %s", hipGetErrorName(e), (int)e, line,
                expr);
  return FAB_E_HIP;
}

#define FAB_TRY(expr)                                              \
  do {                                                             \
    hipError_t e_ = (expr);                                        \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__);    \
  } while (0)

// ---------------------------------------------------------- allocation-free sketch application
// For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc): fab_sketch_apply_noalloc keeps the product kernel's per-block
// partial sketches in `scratch`, a file-scope device array of kMaxParts x kScratchMaxD FP64 (4 MiB),
// instead of a caller's workspace.  Every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names only a stand-in for the symbol: its device address on
// a device comes from hipGetSymbolAddress, taken once per device, with that device current, when
// the first context on it is created (scratch_address), and kept in every context of the device.
constexpr int kScratchMaxD = 256;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[(size_t)kMaxParts * kScratchMaxD];

static hipError_t scratch_address(int device, double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

// Timing events are recorded only on cycles enqueued directly on the stream (timing mode does
// not capture a graph: an event recorded during capture becomes a graph dependency and never
// receives a timestamp, and external event-record nodes are not accepted by this runtime).
static hipError_t record_timing_event(hipEvent_t e, hipStream_t s) { return hipEventRecord(e, s); }

// Enqueue one full cycle (start, m steps, small, optionally pass + convergence test).
// Blocks of the fused SpMV + sketch kernel per member group (gridDim.x; the groups of a batch are
// gridDim.y): as many as are resident on the device at once (the occupancy calculator's count per
// CU, at most 8).  A batch's groups then run in turn, each over a whole wave of blocks, so one
// group's vectors are in flight at a time (sizing gridDim.x to fill the device with all groups at
// once measured slower: 846 against 787 us for 64 members one per block).
static int spmv_grid(const fab_ctx* ctx, int64_t n, int dtype, int mode, int d, int G = 1, int zeta = 1,
                     bool c16 = false) {
  const int per_cu = std::max(1, std::min(8, spmv_blocks_per_cu(dtype, mode, d, G, zeta, c16)));
  return stream_grid(n, std::min(per_cu * ctx->num_cu, kMaxParts));  // one partial per block
}

// Batch geometry: nb members, each with a single-solve workspace bs bytes apart; the fused kernel
// serves G members per block; member r's time points are columns r nt .. r nt + nt - 1 of x.
struct Batch {
  int nb = 1, G = 1;
  size_t bs = 0;
  int64_t ldx = 0;
};

// Sketched methods with zeta <= 8 sketch each cycle's start vector inside the previous cycle's
// pass, so the captured cycle begins without a sketch-only pass over w_1; the solve's set-up
// sketches b for the first cycle (enqueue_first_sketch).
static bool pass_sketches(const fab_params* p) { return p->method != FAB_PLAIN_RESTART && p->zeta <= 8; }

static PassSketch pass_sketch(const fab_params* p, int dtype) {
  PassSketch ps{};
  ps.on = 1;
  ps.d = p->d;
  ps.zeta = p->zeta;
  ps.k0 = (uint32_t)p->seed;
  ps.k1 = (uint32_t)(p->seed >> 32);
  const double sc = 1.0 / std::sqrt((double)p->zeta);
  ps.scale = (dtype == 0) ? sc : (double)(float)sc;  // the sketch-only pass scales by a value of type T
  return ps;
}

static fab_status enqueue_first_sketch(const fab_ctx* ctx, hipStream_t s, const fab_op* A, const fab_params* p,
                                       const Ptrs& q, const Batch& B) {
  if (!pass_sketches(p)) return FAB_OK;
  const int n = (int)A->n;
  const int g_sk = spmv_grid(ctx, n, A->dtype, 1, p->d, B.G, p->zeta);
  FAB_TRY(launch_spmv_sketch(s, A->dtype, 1, g_sk, n, A->rowptr, A->colind, A->colrel, A->vals, q.W, nullptr, p->d,
                             p->zeta, p->seed, q.parts, q.st, B.nb, B.G, B.bs));
  FAB_TRY(launch_reduce_parts(s, 0, p->d, g_sk, q.parts, q.red, q.st, 0, B.nb, B.bs));
  return FAB_OK;
}

static fab_status enqueue_cycle(const fab_ctx* ctx, hipStream_t s, const fab_op* A, const fab_params* p, int fun,
                                int nt, const Layout& L, const Ptrs& q, double* x, Report* rep, bool with_pass,
                                const std::vector<hipEvent_t>* tev, const Batch& B) {
  const int n = (int)A->n, m = p->m, dt = A->dtype;
  const size_t es = dt == 0 ? 8 : 4;
  const bool plain = p->method == FAB_PLAIN_RESTART;
  const int d = plain ? 1 : p->d;
  const int nb = B.nb;
  const size_t bs = B.bs;
  const int g_spmv = spmv_grid(ctx, n, dt, plain ? 2 : 0, d, B.G, p->zeta, A->colrel != nullptr);
  const int g_sk = spmv_grid(ctx, n, dt, 1, d, B.G, p->zeta);
  const int g_vec = stream_grid(n, 2048);
  auto col = [&](int j) -> void* { return (char*)q.W + (size_t)j * wcol(n, (int)es) * es; };
  const bool pass_sk = with_pass && pass_sketches(p);
  if (!plain) {
    if (!pass_sk) {  // otherwise the set-up or the previous cycle's pass formed S w_1 already
      FAB_TRY(launch_spmv_sketch(s, dt, 1, g_sk, n, A->rowptr, A->colind, A->colrel, A->vals, col(0), nullptr, d,
                                 p->zeta, p->seed, q.parts, q.st, nb, B.G, bs));
      FAB_TRY(launch_reduce_parts(s, 0, d, g_sk, q.parts, q.red, q.st, 0, nb, bs));
    }
  } else {
    FAB_TRY(launch_sqnorm(s, dt, g_vec, n, col(0), q.slots_start));
  }
  FAB_TRY(launch_start(s, d, m, plain ? 1 : 0, q.red, q.slots_start, q.slots_step, q.step_len, q.U, q.R, q.st, nb,
                       bs));
  FAB_TRY(launch_scale_col(s, dt, g_vec, n, col(0), &q.st->inv_alpha, q.st, nb, bs));
  // Timing: with events around every kernel (fab_timing_enable(ctx, 1)) the product's and the
  // update's dispatches record them themselves (the kernels' own intervals); with events at the loop
  // ends only (2), one event before the first step and one after the last.
  const bool kev = tev && !ctx->timing_loop_only;
  auto ev = [&](int i) { return kev ? (*tev)[i] : (hipEvent_t) nullptr; };
  if (tev && ctx->timing_loop_only) FAB_TRY(record_timing_event((*tev)[0], s));
  for (int j = 0; j < m; ++j) {
    if (!plain) {
      FAB_TRY(launch_spmv_sketch(s, dt, 0, g_spmv, n, A->rowptr, A->colind, A->colrel, A->vals, col(j), col(j + 1),
                                 d, p->zeta, p->seed, q.parts, q.st, nb, B.G, bs, A->nts, ev(2 * j), ev(2 * j + 1)));
      // Gram-Schmidt folded into the update launch for single solves (every block of the update
      // redoes it; in a batch that redundancy would multiply by the members).  With at most 64
      // product blocks (small operators) the update's Gram-Schmidt wavefront also sums their
      // partial sketches itself, each lane its entries in block order: one launch less per step.
      const bool fused_orth = nb == 1 && d <= 256 && p->k <= 8;
      const bool inline_sum = fused_orth && g_spmv <= 64;
      if (!inline_sum) FAB_TRY(launch_reduce_parts(s, 0, d, g_spmv, q.parts, q.uraw, q.st, 0, nb, bs));
      if (fused_orth) {
        FAB_TRY(launch_orth_update(s, dt, ctx->num_cu, n, j, p->k, m, d, q.W, q.uraw, q.U, q.R, q.G, q.st, nb, bs,
                                   inline_sum ? q.parts : nullptr, inline_sum ? g_spmv : 0, A->nts,
                                   ev(kTevUpdate + 2 * j), ev(kTevUpdate + 2 * j + 1)));
      } else {
        FAB_TRY(launch_orth(s, j, p->k, m, d, q.uraw, q.U, q.R, q.st, nb, bs));
        FAB_TRY(launch_update(s, dt, g_vec, n, j, p->k, q.W, q.st, nb, bs, ev(kTevUpdate + 2 * j),
                              ev(kTevUpdate + 2 * j + 1)));
      }
    } else {
      double* set0 = q.slots_step;
      double* set1 = q.slots_step + q.step_len;
      FAB_TRY(launch_spmv_sketch(s, dt, 2, g_spmv, n, A->rowptr, A->colind, A->colrel, A->vals, col(j), col(j + 1),
                                 1, 1, 0, nullptr, q.st, 1, 1, 0, 0, ev(2 * j), ev(2 * j + 1)));
      FAB_TRY(launch_gram(s, dt, g_vec, n, j + 1, q.W, col(j + 1), set0, 1, q.st));
      FAB_TRY(launch_cgs_update(s, dt, g_vec, n, j, m, q.W, set0, set1, nullptr, 0, q.R, q.st));
      FAB_TRY(launch_gram(s, dt, g_vec, n, j + 1, q.W, col(j + 1), set1, 0, q.st));
      FAB_TRY(launch_cgs_update(s, dt, g_vec, n, j, m, q.W, set1, set0, q.slots_start, 1, q.R, q.st));
      FAB_TRY(launch_plain_finish(s, j, m, q.slots_start, q.R, q.st));
      FAB_TRY(launch_scale_col(s, dt, g_vec, n, col(j + 1), &q.st->inv_rho, q.st, 1, 0));
    }
  }
  if (tev) FAB_TRY(record_timing_event((*tev)[kTevEnd], s));
  SmallArgs a{};
  a.d = d;
  a.m = m;
  a.nt = nt;
  a.plain = plain ? 1 : 0;
  a.fun = fun;
  a.nq = L.nq;
  a.U = q.U;
  a.Uq = q.Ut;
  a.R = q.R;
  a.Tout = q.T;
  a.Xout = q.X;
  a.rz = q.rz;
  a.rw = q.rw;
  a.psi = q.psi;
  a.gbuf = q.gbuf;
  a.C = q.C;
  a.G = q.G;
  a.st = q.st;
  a.bs = bs;
  GrowBuffers gb{};
  if (p->method == FAB_SKETCHED_GROWING) {
    char* g0 = q.base + L.grow;
    gb.M = (double*)g0;
    gb.K = (double*)(g0 + (size_t)kGrowRows * m * 8);
    gb.sz = (int*)(g0 + (size_t)kGrowRows * m * 8 + (size_t)kGrowRows * 8);
    gb.tvals = q.tvals;
  }
  FAB_TRY(launch_small(s, a, nb, p->method == FAB_SKETCHED_GROWING ? &gb : nullptr));
  if (with_pass) {
    // A batch fills the device with its members: fewer, longer blocks (8 elements per thread at
    // n = 1M) spend less on each block's partial norms and bins (64 FP32 members of 1024^2: 6.6%
    // less time per cycle).
    const int g_pass = nb > 1 ? stream_grid(n, 512) : g_vec;
    FAB_TRY(launch_pass(s, dt, g_pass, n, m, nt, d, q.C, q.W, x, B.ldx, q.parts, q.st, nb, bs,
                        pass_sk ? pass_sketch(p, dt) : PassSketch{}));
    // the next start's sketch (entries [0, d)) when the pass formed it, and the norms after it
    if (pass_sk)
      FAB_TRY(launch_reduce_parts(s, 0, d + 2 * nt, g_pass, q.parts, q.red, q.st, 1, nb, bs));
    else
      FAB_TRY(launch_reduce_parts(s, d, 2 * nt, g_pass, q.parts, q.red + d, q.st, 1, nb, bs));
    FAB_TRY(launch_final(s, nt, d, p->tol, ctx->div_limit, dt == 0 ? 0x1p-53 : 0x1p-24, q.red, q.st, rep, nb, bs));
  }
  return FAB_OK;
}

static void info_init(fab_info* h, fab_status s) {
  if (!h) return;
  std::memset(h, 0, sizeof(*h));
  h->status = s;
}

extern "C" {

const char* fab_last_error(void) { return g_last_error; }

const char* fab_status_string(fab_status s) {
  switch (s) {
    case FAB_OK: return "ok";
    case FAB_OK_BREAKDOWN: return "ok: breakdown (invariant subspace, exact result)";
    case FAB_W_NOT_CONVERGED: return "warning: max_cycles reached before the tolerance";
    case FAB_W_QUADRATURE: return "warning: the quadrature rule misses f by more than tol/10 on the spectral region";
    case FAB_E_INVALID: return "error: invalid argument";
    case FAB_E_UNSUPPORTED: return "error: unsupported size or option";
    case FAB_E_HIP: return "error: HIP runtime failure";
    case FAB_E_NONFINITE: return "error: non-finite value in the iteration";
    case FAB_E_DIVERGED: return "error: the restart iteration diverged (increment > 1e8 ||x||)";
    case FAB_E_WORKSPACE: return "error: workspace too small";
  }
  return "unknown status";
}

fab_status fab_create(fab_ctx** ctx, void* hip_stream) {
  if (!ctx) return FAB_E_INVALID;
  *ctx = nullptr;
  fab_ctx* c = new (std::nothrow) fab_ctx();
  if (!c) return FAB_E_HIP;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return FAB_E_HIP;
  }
  c->user = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    c->num_cu = prop.multiProcessorCount;
  }
  if (configure_cycle_kernels() != hipSuccess || configure_step_kernels() != hipSuccess) {
    delete c;
    return FAB_E_HIP;
  }
  {
    const hipError_t e = scratch_address(c->device, &c->scratch);  // the device is current here
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    }
  }
  if (hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&c->h_rep, sizeof(Report) * kMaxBatch, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_t, sizeof(double) * kMaxNt, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&c->d_part, sizeof(double) * kDotBlocks) != hipSuccess) {
    if (c->h_rep) (void)hipHostFree(c->h_rep);
    if (c->h_t) (void)hipHostFree(c->h_t);
    if (c->work) (void)hipStreamDestroy(c->work);
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c;
    return FAB_E_HIP;
  }
  *ctx = c;
  return FAB_OK;
}

fab_status fab_destroy(fab_ctx* c) {
  if (!c) return FAB_E_INVALID;
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto& g : c->ragged_execs) (void)hipGraphExecDestroy(g);
  for (auto& st : c->branch) (void)hipStreamDestroy(st);
  for (auto& e : c->join) (void)hipEventDestroy(e);
  if (c->fork) (void)hipEventDestroy(c->fork);
  for (auto& e : c->tev) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(c->work);
  (void)hipStreamDestroy(c->work);
  (void)hipEventDestroy(c->ev);
  (void)hipHostFree(c->h_rep);
  (void)hipHostFree(c->h_t);
  (void)hipFree(c->d_part);
  delete c;
  return FAB_OK;
}

// Check a new operator's CSR structure on the device (every product indexes with it): row pointers
// non-decreasing from 0 to nnz, column indices in [0, n).  FAB_E_INVALID when it is malformed.
static fab_status validate_op(fab_ctx* ctx, const fab_op* o) {
  hipStream_t s = ctx->work;
  int* dflag = reinterpret_cast<int*>(ctx->d_part);  // the context's reduction buffer, free between calls
  int flag = 0;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));  // the arrays may still be written on the caller's stream
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(hipMemsetAsync(dflag, 0, sizeof(int), s));
  FAB_TRY(launch_csr_validate(s, (int)o->n, (int)o->nnz, o->rowptr, o->colind, dflag));
  FAB_TRY(hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  FAB_TRY(hipStreamSynchronize(s));
  return flag ? FAB_E_INVALID : FAB_OK;
}

// The fused product reads a column index as a 16-bit offset from the first row of its row's
// kThreads-row tile when every column of the matrix lies within [-32768, 32767] of that row
// (matrices of bandwidth below 32K rows, such as grid operators in natural ordering): 10 instead
// of 12 bytes per FP64 nonzero.  The offsets are derived once, from column indices already checked
// to lie in [0, n), so a decoded index stays in range.  Any other matrix, or a failed allocation of
// the 2 bytes per nonzero, leaves colrel null and the product reads colind.
static fab_status derive_col_offsets(fab_ctx* ctx, fab_op* o) {
  if (o->nnz == 0) return FAB_OK;
  int16_t* off = nullptr;
  if (hipMalloc((void**)&off, sizeof(int16_t) * (size_t)o->nnz) != hipSuccess) {
    (void)hipGetLastError();  // out of memory: keep the 32-bit indices
    return FAB_OK;
  }
  hipStream_t s = ctx->work;
  int* dflag = reinterpret_cast<int*>(ctx->d_part);  // the context's reduction buffer, free between calls
  int flag = 0;
  hipError_t e = hipMemsetAsync(dflag, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_col_offsets(s, (int)o->n, o->rowptr, o->colind, off, dflag);
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || flag != 0) {
    (void)hipFree(off);
    return e != hipSuccess ? hip_fail(e, "column offsets", __LINE__) : FAB_OK;
  }
  o->colrel = off;
  return FAB_OK;
}

fab_status fab_csr_create(fab_ctx* ctx, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                          const void* vals, int32_t dtype, fab_op** op) {
  if (!ctx || !op || n <= 0 || nnz < 0 || nnz >= ((int64_t)1 << 31) || !rowptr || (nnz > 0 && (!colind || !vals)))
    return FAB_E_INVALID;
  if (dtype != FAB_F64 && dtype != FAB_F32) return FAB_E_INVALID;
  if (n >= ((int64_t)1 << 31)) return FAB_E_UNSUPPORTED;
  fab_op* o = new (std::nothrow) fab_op{ctx, n, nnz, rowptr, colind, vals, dtype, nullptr, next_op_serial()};
  if (!o) return FAB_E_HIP;
  fab_status st = validate_op(ctx, o);
  if (st == FAB_OK) st = derive_col_offsets(ctx, o);
  if (st != FAB_OK) {
    delete o;
    return st;
  }
  o->nts = size_policy(o);
  *op = o;
  return FAB_OK;
}

fab_status fab_op_destroy(fab_op* op) {
  if (!op) return FAB_E_INVALID;
  if (op->owned) (void)hipFree(op->owned);  // hipFree waits for the device
  if (op->colrel) (void)hipFree(op->colrel);
  delete op;
  return FAB_OK;
}

fab_status fab_op_transpose(fab_ctx* ctx, const fab_op* A, fab_op** AT) {
  if (!ctx || !A || !AT) return FAB_E_INVALID;
  *AT = nullptr;
  const int n = (int)A->n, nnz = (int)A->nnz;
  const size_t es = A->dtype == 0 ? 8 : 4;
  const size_t o_col = align_up(sizeof(int) * ((size_t)n + 1));
  const size_t o_val = o_col + align_up(sizeof(int) * (size_t)std::max(nnz, 1));
  const size_t total = o_val + align_up(es * (size_t)std::max(nnz, 1));
  const size_t nb = transpose_scan_blocks((int64_t)n + 1);
  const size_t t_cur = align_up(sizeof(int) * 64);  // flag at 0, cursor after it, then the scan sums
  const size_t t_sums = t_cur + align_up(sizeof(int) * (size_t)n);
  const size_t ttotal = t_sums + align_up(sizeof(int) * nb);
  char* base = nullptr;
  char* tmp = nullptr;
  hipStream_t s = ctx->work;
  int flag = 0;
  auto fail = [&](hipError_t e, const char* what, int line) {
    if (tmp) (void)hipFree(tmp);
    if (base) (void)hipFree(base);
    return hip_fail(e, what, line);
  };
#define FAB_TRYT(expr)                                               \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) return fail(e_, #expr, __LINE__);          \
  } while (0)
  FAB_TRYT(hipMalloc((void**)&base, total));
  FAB_TRYT(hipMalloc((void**)&tmp, ttotal));
  int* rowptrT = (int*)base;
  int* colT = (int*)(base + o_col);
  void* valT = base + o_val;
  int* dflag = (int*)tmp;
  int* cursor = (int*)(tmp + t_cur);
  int* sums = (int*)(tmp + t_sums);
  FAB_TRYT(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRYT(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRYT(hipMemsetAsync(dflag, 0, sizeof(int), s));
  FAB_TRYT(launch_csr_validate(s, n, nnz, A->rowptr, A->colind, dflag));
  FAB_TRYT(hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  FAB_TRYT(hipStreamSynchronize(s));
  if (flag != 0) {  // every later step indexes with rowptr and colind
    (void)hipFree(tmp);
    (void)hipFree(base);
    return FAB_E_INVALID;
  }
  FAB_TRYT(hipMemsetAsync(rowptrT, 0, sizeof(int) * ((size_t)n + 1), s));
  FAB_TRYT(launch_transpose(s, A->dtype, n, nnz, A->rowptr, A->colind, A->vals, rowptrT, colT, valT, cursor, sums));
  FAB_TRYT(hipStreamSynchronize(s));
#undef FAB_TRYT
  (void)hipFree(tmp);
  fab_op* o = new (std::nothrow) fab_op{ctx, A->n, A->nnz, rowptrT, colT, valT, A->dtype, base, next_op_serial()};
  if (!o) {
    (void)hipFree(base);
    return FAB_E_HIP;
  }
  const fab_status st = derive_col_offsets(ctx, o);
  if (st != FAB_OK) {
    (void)fab_op_destroy(o);
    return st;
  }
  o->nts = size_policy(o);
  *AT = o;
  return FAB_OK;
}

fab_status fab_op_index_bytes(const fab_op* A, int32_t* h_bytes) {
  if (!A || !h_bytes) return FAB_E_INVALID;
  *h_bytes = A->colrel ? 2 : 4;
  return FAB_OK;
}

fab_status fab_op_store_policy(fab_op* A, int32_t policy, int32_t* h_streaming) {
  if (!A || policy < 0 || policy > 2) return FAB_E_INVALID;
  A->nts = policy == 0 ? size_policy(A) : policy - 1;
  if (h_streaming) *h_streaming = A->nts;
  return FAB_OK;
}

fab_status fab_op_copy_arrays(fab_ctx* ctx, const fab_op* A, int32_t* rowptr, int32_t* colind, void* vals) {
  if (!ctx || !A || !rowptr || (A->nnz > 0 && (!colind || !vals))) return FAB_E_INVALID;
  const size_t es = A->dtype == 0 ? 8 : 4;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(hipMemcpyAsync(rowptr, A->rowptr, sizeof(int) * ((size_t)A->n + 1), hipMemcpyDeviceToDevice, s));
  if (A->nnz > 0) {
    FAB_TRY(hipMemcpyAsync(colind, A->colind, sizeof(int) * (size_t)A->nnz, hipMemcpyDeviceToDevice, s));
    FAB_TRY(hipMemcpyAsync(vals, A->vals, es * (size_t)A->nnz, hipMemcpyDeviceToDevice, s));
  }
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_dot(fab_ctx* ctx, int64_t n, const double* x, const double* y, double* out) {
  if (!ctx || !x || !y || !out || n < 0) return FAB_E_INVALID;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(launch_dot(s, n, x, y, ctx->d_part, kDotBlocks, out));
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_workspace_size(const fab_op* A, const fab_params* p, int32_t nt, size_t* h_bytes) {
  if (!A || !p || !h_bytes || nt < 1 || nt > kMaxNt || p->m < 1 || p->m > kMaxM) return FAB_E_INVALID;
  if (p->method == FAB_SKETCHED && (p->d < 1 || p->d > kMaxD)) return FAB_E_INVALID;
  size_t most = 0;  // the largest layout over the functions (they differ in rule nodes)
  for (int fun : {FAB_EXP_NEG, FAB_INVSQRT, FAB_PHI1_NEG, FAB_COS_SQRT})
    most = std::max(most, make_layout(A->n, A->dtype, p, fun, nt).total);
  *h_bytes = most;
  return FAB_OK;
}

fab_status fab_workspace_size_batched(const fab_op* A, const fab_params* p, int32_t nt, int32_t nb, size_t* h_bytes) {
  if (nb < 1 || nb > kMaxBatch) return FAB_E_INVALID;
  size_t one = 0;
  const fab_status st = fab_workspace_size(A, p, nt, &one);
  if (st != FAB_OK) return st;
  *h_bytes = (nb == 1) ? one : (size_t)nb * align_up(one);
  return FAB_OK;
}

// Members per block of the fused SpMV + sketch kernel for a batch: each candidate is timed on the
// batch's own operator and workspace (HIP events, 3 launches after 1 warm-up) and the fastest is
// kept for this operator and batch shape.  Runs before the solve's set-up, which clears what the
// timing launches wrote.
// Whether the grouped kernel can serve G members per block: its dynamic LDS (G d FP64 bins, the
// tile's table of S, the CSR chunk) within what configure_step_kernels allows, and each member's
// vector addressable as one buffer (n times the value size below 2^31 bytes).
static bool group_fits(int dtype, int64_t n, const fab_params* p, int G) {
  return n * (dtype == 0 ? 8 : 4) <= INT32_MAX && spmv_sketch_lds(dtype, 0, p->d, G, p->zeta, false) <= group_lds_max() &&
         spmv_sketch_lds(dtype, 1, p->d, G, p->zeta, false) <= group_lds_max();
}

static fab_status tune_group(fab_ctx* ctx, const fab_op* A, const fab_params* p, int nb, const Ptrs& q, size_t bs,
                             int* G_out) {
  *G_out = 1;
  if (nb <= 1 || p->method == FAB_PLAIN_RESTART) return FAB_OK;
  if (ctx->force_group > 0) {  // a forced group the grouped kernel cannot serve falls back to 1
    *G_out = (ctx->force_group > 1 && !group_fits(A->dtype, A->n, p, ctx->force_group)) ? 1 : ctx->force_group;
    return FAB_OK;
  }
  for (const auto& t : ctx->tuned)
    if (t.op == A->serial && t.n == A->n && t.nb == nb && t.d == p->d && t.zeta == p->zeta && t.dtype == A->dtype) {
      *G_out = t.G;
      return FAB_OK;
    }
  const int n = (int)A->n, dt = A->dtype, d = p->d;
  const size_t es = dt == 0 ? 8 : 4;
  hipStream_t s = ctx->work;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  FAB_TRY(hipEventCreate(&e0));
  FAB_TRY(hipEventCreate(&e1));
  int best = 1;
  float best_ms = 1e30f;
  hipError_t err = hipSuccess;
  // candidates: one member per block, or groups of 4, 8 or 16 (one to four members per wavefront;
  // padding members past nb cost nothing)
  for (int G = 1; G <= 16 && err == hipSuccess; G = (G == 1 ? 4 : 2 * G)) {
    if (G > 1 && (!group_fits(dt, A->n, p, G) || G > 4 * nb)) break;
    const int grid = spmv_grid(ctx, n, dt, 0, d, G, p->zeta, A->colrel != nullptr);
    void* x0 = q.W;
    void* y0 = (char*)q.W + wcol(n, (int)es) * es;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
      if (rep == 1) err = hipEventRecord(e0, s);
      if (err == hipSuccess)
        err = launch_spmv_sketch(s, dt, 0, grid, n, A->rowptr, A->colind, A->colrel, A->vals, x0, y0, d, p->zeta,
                                 p->seed, q.parts, nullptr, nb, G, bs);
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = G;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(err, "tune_group", __LINE__);
  if (ctx->tuned.size() >= 64) ctx->tuned.erase(ctx->tuned.begin());  // oldest first
  ctx->tuned.push_back({A->serial, A->n, nb, d, p->zeta, A->dtype, best});
  *G_out = best;
  return FAB_OK;
}

static int status_rank(fab_status s) { return s < 0 ? 100 - (int)s : (int)s; }  // errors above warnings

// Per-member outcome of the restarted loop, updated from each cycle's report.
struct Track {
  fab_status status = FAB_W_NOT_CONVERGED;
  int cycles = 0, matvecs = 0;
  bool finished = false;
  double est = 0.0, err_est = 0.0, rule_err = 0.0, kappa_T = 1.0;
};

// Returns true when this report finishes the member.
static bool track_report(Track& t, const Report& rr, int c, double div_limit) {
  t.cycles = c + 1;
  t.matvecs += rr.meff;
  t.est = rr.relupd;
  t.err_est = rr.est;
  t.rule_err = std::max(t.rule_err, rr.rule_err);
  if (rr.meff > 0 && std::isfinite(rr.kappa_T)) t.kappa_T = std::max(t.kappa_T, rr.kappa_T);
  if (rr.nonfinite) {
    t.status = FAB_E_NONFINITE;
  } else if (rr.grow_fail) {  // growing restart out of capacity or Taylor steps
    t.status = FAB_E_UNSUPPORTED;
  } else if (rr.brk) {
    t.status = (rr.meff == 0 && c == 0) ? FAB_OK : FAB_OK_BREAKDOWN;  // b = 0: x = 0 exactly
  } else if (rr.converged) {
    t.status = FAB_OK;
  } else if (!(rr.relupd <= div_limit)) {
    // Transient growth of the increments (est ~ 1) is normal on wide spectra: the restarted
    // iteration of a fixed rule still converges.  Only increments that dwarf the iterate stop it.
    t.status = FAB_E_DIVERGED;
  } else {
    return false;
  }
  t.finished = true;
  return true;
}

// Final statuses into h_info; returns the most severe.
static fab_status finish_tracks(std::vector<Track>& tr, const fab_params* p, fab_info* h_info, int group) {
  fab_status worst = FAB_OK;
  for (size_t r = 0; r < tr.size(); ++r) {
    Track& t = tr[r];
    // A fixed rule r makes the restarted iteration converge to r(A) b, so the rule adds at most its
    // error |r - f| over the spectral region to the result (k_rule_check samples it once per solve).
    if (p->method == FAB_SKETCHED_GROWING) t.rule_err = 0.0;  // no quadrature rule in this restart
    if ((t.status == FAB_OK || t.status == FAB_OK_BREAKDOWN) && t.rule_err > std::max(0.1 * p->tol, 1e-11))
      t.status = FAB_W_QUADRATURE;
    if (status_rank(t.status) > status_rank(worst)) worst = t.status;
    if (h_info) {
      h_info[r].status = t.status;
      h_info[r].cycles = t.cycles;
      h_info[r].matvecs = t.matvecs;
      h_info[r].est_rel_update = t.est;
      h_info[r].err_est = t.err_est;
      h_info[r].quad_rule_error = t.rule_err;
      h_info[r].kappa_T = t.kappa_T;
      h_info[r].group = group;
    }
  }
  return worst;
}

// The restarted loop of Algorithm 2 for nb right-hand sides (columns of b, leading dimension ldb)
// sharing A; member r's result for time point i is column r nt + i of x (leading dimension ldx).
static fab_status solve_batch(fab_ctx* ctx, const fab_op* A, int32_t fun, const double* h_t, int32_t nt, int nb,
                              const void* b, int64_t ldb, double* x, int64_t ldx, const fab_params* p, void* work,
                              size_t work_bytes, fab_info* h_info) {
  for (int r = 0; r < nb; ++r) info_init(h_info ? h_info + r : nullptr, FAB_E_INVALID);
  if (!ctx || !A || !b || !x || !p || !work) return FAB_E_INVALID;
  if (nb < 1 || nb > kMaxBatch || ldb < A->n || ldx < A->n) return FAB_E_INVALID;
  if (nb > 1 && p->method != FAB_SKETCHED) {  // batches run the sketched method with the quadrature restart
    for (int r = 0; r < nb; ++r) info_init(h_info ? h_info + r : nullptr, FAB_E_UNSUPPORTED);
    return FAB_E_UNSUPPORTED;
  }
  if (timed_fun(fun) && !h_t) return FAB_E_INVALID;
  fab_status ps = check_params(A, p, fun, nt);
  if (ps != FAB_OK) {
    for (int r = 0; r < nb; ++r) info_init(h_info ? h_info + r : nullptr, ps);
    return ps;
  }
  if (timed_fun(fun))
    for (int i = 0; i < nt; ++i)
      if (!std::isfinite(h_t[i]) || !(h_t[i] > 0.0)) return FAB_E_INVALID;
  if (((uintptr_t)work & 255) != 0) return FAB_E_INVALID;
  const Layout L = make_layout(A->n, A->dtype, p, fun, nt);
  const size_t bs = (nb == 1) ? 0 : align_up(L.total);
  const size_t need = (nb == 1) ? L.total : (size_t)nb * bs;
  if (work_bytes < need) {
    for (int r = 0; r < nb; ++r) info_init(h_info ? h_info + r : nullptr, FAB_E_WORKSPACE);
    return FAB_E_WORKSPACE;
  }
  for (int r = 0; r < nb; ++r) info_init(h_info ? h_info + r : nullptr, FAB_E_HIP);
  const Ptrs q = carve(work, L, p, nt);
  hipStream_t s = ctx->work;
  const int n = (int)A->n;
  // order after the caller's stream
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  Batch B;
  B.nb = nb;
  B.bs = bs;
  B.ldx = ldx;
  const fab_status ts = tune_group(ctx, A, p, nb, q, bs, &B.G);
  if (ts != FAB_OK) return ts;
  // solve set-up: zero accumulators, state and x; quadrature nodes; w_1 <- b
  FAB_TRY(launch_zero_strided(s, (double*)((char*)work + L.slots_step), (L.T - L.slots_step) / 8, nb, bs));
  FAB_TRY(launch_zero_strided(s, x, (size_t)n, nb * nt, (size_t)ldx * 8));
  FAB_TRY(hipStreamSynchronize(s));  // the pinned staging buffer may still feed a previous call
  for (int i = 0; i < nt; ++i) ctx->h_t[i] = timed_fun(fun) ? h_t[i] : 1.0;
  FAB_TRY(hipMemcpyAsync(q.tvals, ctx->h_t, sizeof(double) * nt, hipMemcpyHostToDevice, s));
  FAB_TRY(launch_rule(s, fun, nt, q.tvals, rule_nodes(fun, p), p->spec_lo, p->spec_hi, q.rz, q.rw, q.psi, q.st, nb,
                      bs));
  FAB_TRY(launch_copy_in(s, A->dtype, stream_grid(n, 2048), n, b, ldb, q.W, nb, bs));
  {
    const fab_status fs = enqueue_first_sketch(ctx, s, A, p, q, B);
    if (fs != FAB_OK) return fs;
  }

  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.op = A->serial;
  key.work = work;
  key.x = x;
  key.n = A->n;
  key.m = p->m;
  key.k = p->k;
  key.d = p->d;
  key.zeta = p->zeta;
  key.nt = nt;
  key.fun = fun;
  key.method = p->method;
  key.nq = rule_nodes(fun, p);
  key.dtype = A->dtype;
  key.seed = p->seed;
  key.tol = p->tol;
  key.nb = nb;
  key.G = B.G;
  key.ldx = ldx;
  key.bs = bs;
  key.div_limit = ctx->div_limit;
  key.nts = A->nts;
  hipGraphExec_t exec = nullptr;
  for (auto& g : ctx->graphs)
    if (g.key == key) exec = g.exec;
  if (!exec && !ctx->timing) {
    hipGraph_t graph;
    FAB_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    fab_status es = enqueue_cycle(ctx, s, A, p, fun, nt, L, q, x, ctx->h_rep, true, nullptr, B);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (es != FAB_OK) return es;
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture", __LINE__);
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate", __LINE__);
    if (ctx->graphs.size() >= 8) {
      (void)hipGraphExecDestroy(ctx->graphs.front().exec);
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({key, exec});
  }
  std::vector<Track> tr(nb);
  int remaining = nb;
  for (int c = 0; c < p->max_cycles && remaining > 0; ++c) {
    if (ctx->timing) {
      const fab_status es = enqueue_cycle(ctx, s, A, p, fun, nt, L, q, x, ctx->h_rep, true, &ctx->tev, B);
      if (es != FAB_OK) return es;
    } else {
      FAB_TRY(hipGraphLaunch(exec, s));
    }
    FAB_TRY(hipStreamSynchronize(s));
    int steps = 0;  // steps run this cycle: the longest among members still iterating
    for (int r = 0; r < nb; ++r) {
      if (tr[r].finished) continue;
      const Report rr = ctx->h_rep[r];
      if (!rr.nonfinite) steps = std::max(steps, rr.meff);
      if (track_report(tr[r], rr, c, ctx->div_limit)) --remaining;
    }
    if (ctx->timing) {
      // the update of a step runs when the step does not break down: the steps before the last
      // always, the last one only for a full cycle (the sketched path; the plain comparator records none)
      const int upd = (p->method == FAB_PLAIN_RESTART || ctx->timing_loop_only)
                          ? 0
                          : (steps == p->m ? steps : std::max(steps - 1, 0));
      for (int j = 0; j < steps && !ctx->timing_loop_only; ++j) {
        float ms = 0.f;
        FAB_TRY(hipEventElapsedTime(&ms, ctx->tev[2 * j], ctx->tev[2 * j + 1]));
        ctx->t_spmv_ms += ms;
      }
      for (int j = 0; j < upd; ++j) {
        float ms = 0.f;
        FAB_TRY(hipEventElapsedTime(&ms, ctx->tev[kTevUpdate + 2 * j], ctx->tev[kTevUpdate + 2 * j + 1]));
        ctx->t_upd_ms += ms;
      }
      ctx->t_spmv_n += ctx->timing_loop_only ? 0 : steps;
      ctx->t_upd_n += upd;
      if (steps == p->m) {
        float ms = 0.f;
        FAB_TRY(hipEventElapsedTime(&ms, ctx->tev[0], ctx->tev[kTevEnd]));
        ctx->t_loop_ms += ms;
        ctx->t_loop_n += steps;
      }
    }
  }
  return finish_tracks(tr, p, h_info, B.G);
}

// ----------------------------------------------------------------------------- ragged batches
constexpr int kBranches = 16;  // branch streams of the ragged graphs (one replayed solve of 32
                                // operators: 50 ms with 4, 37 with 8, 31 with 16 and with 32)

fab_status fab_workspace_size_ragged(int32_t nops, const fab_op* const* ops, const fab_params* p, int32_t nt,
                                     size_t* h_bytes) {
  if (!ops || !p || !h_bytes || nops < 1 || nops > kMaxBatch) return FAB_E_INVALID;
  size_t total = 0;
  for (int i = 0; i < nops; ++i) {
    if (!ops[i]) return FAB_E_INVALID;
    size_t one = 0;
    const fab_status st = fab_workspace_size(ops[i], p, nt, &one);
    if (st != FAB_OK) return st;
    total += align_up(one);
  }
  *h_bytes = total;
  return FAB_OK;
}

// Operators of uneven size, one right-hand side each: every operator runs the single-solve cycle in
// its own workspace; the cycles of all operators are captured once, on kBranches forked streams,
// into one graph that is replayed once per cycle (finished operators' kernels return at once).
fab_status fab_solve_ragged(fab_ctx* ctx, int32_t nops, const fab_op* const* ops, int32_t fun, const double* h_t,
                            int32_t nt, const void* const* b, double* const* x, const fab_params* p, void* work,
                            size_t work_bytes, fab_info* h_info) {
  for (int i = 0; i < nops && h_info; ++i) info_init(h_info + i, FAB_E_INVALID);
  if (!ctx || !ops || !b || !x || !p || !work || nops < 1 || nops > kMaxBatch) return FAB_E_INVALID;
  if (p->method != FAB_SKETCHED) return FAB_E_UNSUPPORTED;
  if (timed_fun(fun) && !h_t) return FAB_E_INVALID;
  if (((uintptr_t)work & 255) != 0) return FAB_E_INVALID;
  for (int i = 0; i < nops; ++i) {
    if (!ops[i] || !b[i] || !x[i]) return FAB_E_INVALID;
    const fab_status ps = check_params(ops[i], p, fun, nt);
    if (ps != FAB_OK) return ps;
  }
  if (timed_fun(fun))
    for (int i = 0; i < nt; ++i)
      if (!std::isfinite(h_t[i]) || !(h_t[i] > 0.0)) return FAB_E_INVALID;
  size_t need = 0;
  if (fab_workspace_size_ragged(nops, ops, p, nt, &need) != FAB_OK) return FAB_E_INVALID;
  if (work_bytes < need) {
    for (int i = 0; i < nops && h_info; ++i) info_init(h_info + i, FAB_E_WORKSPACE);
    return FAB_E_WORKSPACE;
  }
  for (int i = 0; i < nops && h_info; ++i) info_init(h_info + i, FAB_E_HIP);
  std::vector<Layout> L(nops);
  std::vector<Ptrs> q(nops);
  size_t off = 0;
  for (int i = 0; i < nops; ++i) {
    L[i] = make_layout(ops[i]->n, ops[i]->dtype, p, fun, nt);
    q[i] = carve((char*)work + off, L[i], p, nt);
    size_t one = 0;
    (void)fab_workspace_size(ops[i], p, nt, &one);
    off += align_up(one);
  }
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(hipStreamSynchronize(s));  // the pinned staging buffer may still feed a previous call
  for (int i = 0; i < nt; ++i) ctx->h_t[i] = timed_fun(fun) ? h_t[i] : 1.0;
  for (int i = 0; i < nops; ++i) {  // per-operator set-up, as in a single solve
    const int n = (int)ops[i]->n;
    FAB_TRY(launch_zero(s, (double*)((char*)q[i].base + L[i].slots_step), (L[i].T - L[i].slots_step) / 8));
    FAB_TRY(launch_zero(s, x[i], (size_t)n * nt));
    FAB_TRY(hipMemcpyAsync(q[i].tvals, ctx->h_t, sizeof(double) * nt, hipMemcpyHostToDevice, s));
    FAB_TRY(launch_rule(s, fun, nt, q[i].tvals, rule_nodes(fun, p), p->spec_lo, p->spec_hi, q[i].rz, q[i].rw,
                        q[i].psi, q[i].st, 1, 0));
    FAB_TRY(launch_copy_in(s, ops[i]->dtype, stream_grid(n, 2048), n, b[i], n, q[i].W, 1, 0));
    const fab_status fs = enqueue_first_sketch(ctx, s, ops[i], p, q[i], Batch{});
    if (fs != FAB_OK) return fs;
  }
  const int nbr = std::min(nops, kBranches);
  while ((int)ctx->branch.size() < kBranches) {
    hipStream_t bs_ = nullptr;
    hipEvent_t je = nullptr;
    FAB_TRY(hipStreamCreateWithFlags(&bs_, hipStreamNonBlocking));
    FAB_TRY(hipEventCreateWithFlags(&je, hipEventDisableTiming));
    ctx->branch.push_back(bs_);
    ctx->join.push_back(je);
  }
  if (!ctx->fork) FAB_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  std::vector<uintptr_t> key = {(uintptr_t)nops, (uintptr_t)fun, (uintptr_t)nt, (uintptr_t)work,
                                (uintptr_t)p->m, (uintptr_t)p->k, (uintptr_t)p->d, (uintptr_t)p->zeta,
                                (uintptr_t)p->seed, (uintptr_t)rule_nodes(fun, p)};
  uint64_t tolbits, divbits;
  std::memcpy(&tolbits, &p->tol, 8);
  std::memcpy(&divbits, &ctx->div_limit, 8);
  key.push_back((uintptr_t)tolbits);
  key.push_back((uintptr_t)divbits);
  for (int i = 0; i < nops; ++i) {  // operators by serial: a destroyed operator's address can be reused
    key.push_back((uintptr_t)ops[i]->serial);
    key.push_back((uintptr_t)ops[i]->nts);
    key.push_back((uintptr_t)x[i]);
  }
  auto cycle_of = [&](int i, hipStream_t st) {
    Batch B;
    B.ldx = ops[i]->n;
    return enqueue_cycle(ctx, st, ops[i], p, fun, nt, L[i], q[i], x[i], ctx->h_rep + i, true, nullptr, B);
  };
  // The context's first ragged call captures its graphs, one per branch stream (branch j: the
  // cycles of operators j, j + nbr, ... in turn), and calls with the same key replay them, each
  // branch on its own stream between a fork and a join event.  (One graph whose branches were
  // forked inside it took 67 ms per solve of 32 operators, these graphs 31 ms on 16 streams.)  A call with
  // another key does not replace the graphs: its cycles run uncaptured,
  // one operator after another on the work stream, as in timing mode.  (Replacing the graph, a new
  // capture over the same branch streams and fork/join events, is the call in which a host
  // segmentation fault was seen once, with its cause not found; that path is switched off.)
  const bool eager = ctx->timing || (!ctx->ragged_execs.empty() && key != ctx->ragged_key);
  if (!eager && ctx->ragged_execs.empty()) {
    std::vector<hipGraphExec_t> execs;
    auto drop = [&execs]() {
      for (auto& g : execs) (void)hipGraphExecDestroy(g);
    };
    for (int j = 0; j < nbr; ++j) {
      hipStream_t bst = ctx->branch[j];
      const hipError_t be = hipStreamBeginCapture(bst, hipStreamCaptureModeThreadLocal);
      if (be != hipSuccess) {
        drop();
        return hip_fail(be, "hipStreamBeginCapture", __LINE__);
      }
      fab_status es = FAB_OK;
      for (int i = j; i < nops && es == FAB_OK; i += nbr) es = cycle_of(i, bst);
      hipGraph_t graph = nullptr;
      const hipError_t ce = hipStreamEndCapture(bst, &graph);  // always end the capture
      if (es != FAB_OK || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        drop();
        return es != FAB_OK ? es : hip_fail(ce, "hipStreamEndCapture", __LINE__);
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        drop();
        return hip_fail(ie, "hipGraphInstantiate", __LINE__);
      }
      execs.push_back(ex);
    }
    ctx->ragged_execs = std::move(execs);
    ctx->ragged_key = key;
  }
  std::vector<Track> tr(nops);
  int remaining = nops;
  for (int c = 0; c < p->max_cycles && remaining > 0; ++c) {
    if (eager) {  // the same cycles enqueued one operator after another
      for (int i = 0; i < nops; ++i) {
        const fab_status es = cycle_of(i, s);
        if (es != FAB_OK) return es;
      }
    } else {
      FAB_TRY(hipEventRecord(ctx->fork, s));
      for (int j = 0; j < nbr; ++j) {
        FAB_TRY(hipStreamWaitEvent(ctx->branch[j], ctx->fork, 0));
        FAB_TRY(hipGraphLaunch(ctx->ragged_execs[j], ctx->branch[j]));
        FAB_TRY(hipEventRecord(ctx->join[j], ctx->branch[j]));
        FAB_TRY(hipStreamWaitEvent(s, ctx->join[j], 0));
      }
    }
    FAB_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < nops; ++i)
      if (!tr[i].finished && track_report(tr[i], ctx->h_rep[i], c, ctx->div_limit)) --remaining;
  }
  return finish_tracks(tr, p, h_info, 1);
}

fab_status fab_solve(fab_ctx* ctx, const fab_op* A, int32_t fun, const double* h_t, int32_t nt, const void* b,
                     double* x, const fab_params* p, void* work, size_t work_bytes, fab_info* h_info) {
  if (!A) {
    info_init(h_info, FAB_E_INVALID);
    return FAB_E_INVALID;
  }
  return solve_batch(ctx, A, fun, h_t, nt, 1, b, A->n, x, A->n, p, work, work_bytes, h_info);
}

fab_status fab_solve_batched(fab_ctx* ctx, const fab_op* A, int32_t fun, const double* h_t, int32_t nt, int32_t nb,
                             const void* b, int64_t ldb, double* x, int64_t ldx, const fab_params* p, void* work,
                             size_t work_bytes, fab_info* h_info) {
  return solve_batch(ctx, A, fun, h_t, nt, nb, b, ldb, x, ldx, p, work, work_bytes, h_info);
}

fab_status fab_divergence_limit(fab_ctx* ctx, double limit) {
  if (!ctx || !(limit > 0.0)) return FAB_E_INVALID;
  ctx->div_limit = limit;
  return FAB_OK;
}

fab_status fab_batch_group(fab_ctx* ctx, int32_t G) {
  if (!ctx || (G != 0 && G != 1 && G != 4 && G != 8 && G != 16)) return FAB_E_INVALID;
  ctx->force_group = G;
  return FAB_OK;
}

fab_status fab_timing_enable(fab_ctx* ctx, int32_t on) {
  if (!ctx) return FAB_E_INVALID;
  if (on && ctx->tev.empty()) {
    ctx->tev.resize(kTevEnd + 1, nullptr);
    for (auto& e : ctx->tev)
      if (hipEventCreate(&e) != hipSuccess) return FAB_E_HIP;
  }
  if (on < 0 || on > 2) return FAB_E_INVALID;
  ctx->timing = on != 0;
  ctx->timing_loop_only = on == 2;
  ctx->t_spmv_ms = ctx->t_loop_ms = ctx->t_upd_ms = 0.0;
  ctx->t_spmv_n = ctx->t_loop_n = ctx->t_upd_n = 0;
  return FAB_OK;
}

fab_status fab_timing_read(fab_ctx* ctx, double* h_spmv_ms, int64_t* h_spmv_launches, double* h_loop_ms,
                           int64_t* h_loop_steps, double* h_update_ms, int64_t* h_update_launches) {
  if (!ctx || !h_spmv_ms || !h_spmv_launches || !h_loop_ms || !h_loop_steps || !h_update_ms || !h_update_launches)
    return FAB_E_INVALID;
  *h_spmv_ms = ctx->t_spmv_ms;
  *h_spmv_launches = ctx->t_spmv_n;
  *h_loop_ms = ctx->t_loop_ms;
  *h_loop_steps = ctx->t_loop_n;
  *h_update_ms = ctx->t_upd_ms;
  *h_update_launches = ctx->t_upd_n;
  ctx->t_spmv_ms = ctx->t_loop_ms = ctx->t_upd_ms = 0.0;
  ctx->t_spmv_n = ctx->t_loop_n = ctx->t_upd_n = 0;
  return FAB_OK;
}

fab_status fab_spmv(fab_ctx* ctx, const fab_op* A, const void* x, void* y, void* work, size_t work_bytes) {
  (void)work;
  (void)work_bytes;
  if (!ctx || !A || !x || !y) return FAB_E_INVALID;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(launch_spmv_sketch(s, A->dtype, 2, spmv_grid(ctx, A->n, A->dtype, 2, 1, 1, 1, A->colrel != nullptr), (int)A->n, A->rowptr, A->colind,
                             A->colrel, A->vals, x, y, 1, 1, 0, nullptr, nullptr, 1, 1, 0));
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_sketch_apply(fab_ctx* ctx, int64_t n, int32_t d, int32_t zeta, uint64_t seed, int32_t dtype,
                            const void* x, double* Sx, void* work, size_t work_bytes) {
  if (!ctx || !x || !Sx || !work || n <= 0 || n >= ((int64_t)1 << 31) || d < 1 || d > kMaxD || zeta < 1 ||
      zeta > 32 || zeta > d || (dtype != FAB_F64 && dtype != FAB_F32))
    return FAB_E_INVALID;
  if (work_bytes < (size_t)kMaxParts * d * 8) return FAB_E_WORKSPACE;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  double* parts = (double*)work;
  const int grid = spmv_grid(ctx, n, dtype, 1, d, 1, zeta);
  FAB_TRY(launch_spmv_sketch(s, dtype, 1, grid, (int)n, nullptr, nullptr, nullptr, nullptr, x, nullptr, d, zeta, seed,
                             parts, nullptr, 1, 1, 0));
  FAB_TRY(launch_reduce_parts(s, 0, d, grid, parts, Sx, nullptr, -1, 1, 0));
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_sketch_apply_noalloc(fab_ctx* ctx, int64_t n, int32_t d, int32_t zeta, uint64_t seed, int32_t dtype,
                                    const void* x, double* Sx) {
  if (!ctx || !x || !Sx || n <= 0 || n >= ((int64_t)1 << 31) || d < 1 || zeta < 1 || zeta > 32 || zeta > d ||
      (dtype != FAB_F64 && dtype != FAB_F32))
    return FAB_E_INVALID;
  if (d > kScratchMaxD) return FAB_E_UNSUPPORTED;  // beyond the static scratch
  if (!ctx->scratch) return FAB_E_HIP;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  // the same kernels and grid as fab_sketch_apply; every block overwrites its partial (rows
  // [0, d) x the grid), so nothing in scratch needs clearing
  const int grid = spmv_grid(ctx, n, dtype, 1, d, 1, zeta);
  FAB_TRY(launch_spmv_sketch(s, dtype, 1, grid, (int)n, nullptr, nullptr, nullptr, nullptr, x, nullptr, d, zeta, seed,
                             ctx->scratch, nullptr, 1, 1, 0));
  FAB_TRY(launch_reduce_parts(s, 0, d, grid, ctx->scratch, Sx, nullptr, -1, 1, 0));
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_sketch_table(fab_ctx* ctx, int64_t col0, int64_t count, int32_t d, int32_t zeta, uint64_t seed,
                            int32_t* rows, int8_t* signs) {
  if (!ctx || !rows || !signs || col0 < 0 || count < 1 || d < 1 || d > kMaxD || zeta < 1 || zeta > 32 || zeta > d)
    return FAB_E_INVALID;
  hipStream_t s = ctx->work;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(launch_sketch_table(s, col0, count, d, zeta, seed, rows, signs));
  FAB_TRY(hipStreamSynchronize(s));
  return FAB_OK;
}

fab_status fab_cycle_debug(fab_ctx* ctx, const fab_op* A, const void* v, const fab_params* p, void* W, double* U,
                           double* R, double* T, double* X, double* h_scal, void* work, size_t work_bytes) {
  if (!ctx || !A || !v || !p || !W || !U || !R || !T || !X || !h_scal || !work) return FAB_E_INVALID;
  fab_status ps = check_params(A, p, FAB_EXP_NEG, 1);
  if (ps != FAB_OK) return ps;
  const Layout L = make_layout(A->n, A->dtype, p, FAB_EXP_NEG, 1);
  if (work_bytes < L.total) return FAB_E_WORKSPACE;
  const Ptrs q = carve(work, L, p, 1);
  hipStream_t s = ctx->work;
  const int n = (int)A->n, m = p->m;
  const bool plain = p->method == FAB_PLAIN_RESTART;
  const int d = plain ? 1 : p->d;
  const size_t es = A->dtype == 0 ? 8 : 4;
  FAB_TRY(hipEventRecord(ctx->ev, ctx->user));
  FAB_TRY(hipStreamWaitEvent(s, ctx->ev, 0));
  FAB_TRY(launch_zero(s, (double*)((char*)work + L.slots_step), (L.T - L.slots_step) / 8));
  FAB_TRY(hipStreamSynchronize(s));
  ctx->h_t[0] = 1.0;
  FAB_TRY(hipMemcpyAsync(q.tvals, ctx->h_t, sizeof(double), hipMemcpyHostToDevice, s));
  FAB_TRY(launch_rule(s, FAB_EXP_NEG, 1, q.tvals, rule_nodes(FAB_EXP_NEG, p), 0.0, 0.0, q.rz, q.rw, q.psi, q.st, 1,
                      0));
  FAB_TRY(launch_copy_in(s, A->dtype, stream_grid(n, 2048), n, v, n, q.W, 1, 0));
  fab_status es2 = enqueue_cycle(ctx, s, A, p, FAB_EXP_NEG, 1, L, q, nullptr, nullptr, false, nullptr, Batch{});
  if (es2 != FAB_OK) return es2;
  FAB_TRY(hipMemcpy2DAsync(W, (size_t)n * es, q.W, wcol(n, (int)es) * es, (size_t)n * es, m + 1,
                           hipMemcpyDeviceToDevice, s));
  if (!plain) FAB_TRY(hipMemcpyAsync(U, q.U, (size_t)d * (m + 1) * 8, hipMemcpyDeviceToDevice, s));
  FAB_TRY(hipMemcpyAsync(R, q.R, (size_t)(m + 1) * m * 8, hipMemcpyDeviceToDevice, s));
  FAB_TRY(hipMemcpyAsync(T, q.T, (size_t)(m + 1) * (m + 1) * 8, hipMemcpyDeviceToDevice, s));
  FAB_TRY(hipMemcpyAsync(X, q.X, (size_t)m * m * 8, hipMemcpyDeviceToDevice, s));
  State hst;
  FAB_TRY(hipMemcpyAsync(&hst, q.st, sizeof(State), hipMemcpyDeviceToHost, s));
  FAB_TRY(hipStreamSynchronize(s));
  h_scal[0] = hst.alpha;
  h_scal[1] = hst.beta;
  h_scal[2] = hst.h;
  h_scal[3] = (double)hst.meff;
  h_scal[4] = (double)hst.whiten_chol;
  return hst.nonfinite ? FAB_E_NONFINITE : FAB_OK;
}

}  // extern "C"
